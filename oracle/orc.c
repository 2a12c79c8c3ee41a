/*
 * orc.c -- plain FP64 CPU oracle of the settling-particle time step of
 * arXiv 2408.15115 ("Palabos Turret").
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
 * CPU-baseline leg load this library; the product library never does, and
 * this file shares no code, header, table or helper with it.
 *
 * It is deliberately slow and literal: every formula is the one printed in
 * the paper, evaluated in double precision, in the paper's order:
 *
 *   lattice ........ Sec. 2.1, D3Q27 velocity-set equation (k,l,m read as -1,0,1)
 *   moments ........ Sec. 2.1, equations for p and u
 *   equilibrium .... App. A, D3Q27 f^(0) (Hermite sum, all printed terms)
 *   off-equilibrium  App. A, D3Q27 f^(1) and the recursion for a_1^(n)
 *   collision ...... Sec. 2.1 evolution rule, Sec. 2.2 forced evolution rule
 *   stress ......... Sec. 2.1, stress tensor from populations
 *   weight function  Sec. 2.2, W and the one-dimensional w(r)
 *   multi-direct IBM Sec. 2.2, steps l = 0..4, n = 4 cycles
 *   force / torque . Sec. 2.2, stress integral over the markers
 *   rigid body ..... Sec. 2.3, leapfrog with the orientation predictor-corrector
 *   time iteration . Sec. 2.4, Table 1 events (1)-(4)
 *   re-injection ... Sec. 2.5 (falling-frame window)
 *
 * Readings where the paper is silent or garbled are listed at the functions
 * that take them.  Lattice units throughout: dx = dt = rho_0 = rho_f = 1.
 *
 * Grid layout (oracle-private): cell = x + nx*(y + ny*z), populations
 * f[cell*27 + i].  Direction i = 9*(xi_z+1) + 3*(xi_y+1) + (xi_x+1).
 * The vertical axis is z; gravity points along -z.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define Q 27
#define CS2 (1.0 / 3.0)
#define RHO0 1.0

/* ---------------------------------------------------------------- lattice */

static int g_xi[Q][3];
static double g_w[Q];
static int g_ready = 0;

/* Hermite tensor polynomial H^(n)_{al_0..al_{n-1}}(xi) of the Gaussian weight
 * with variance cs^2, from the textbook three-term recurrence
 *   H^(n)_{a,b} = xi_b H^(n-1)_a - cs^2 sum_j delta_{a_j b} H^(n-2)_{a without a_j}. */
static double hermite(const int xi[3], const int *al, int n)
{
    if (n == 0) return 1.0;
    int last = al[n - 1];
    double s = xi[last] * hermite(xi, al, n - 1);
    int sub[8];
    for (int j = 0; j < n - 1; j++) {
        if (al[j] != last) continue;
        int m = 0;
        for (int k = 0; k < n - 1; k++)
            if (k != j) sub[m++] = al[k];
        s -= CS2 * hermite(xi, sub, n - 2);
    }
    return s;
}

/* The printed terms of orders 3..6 of App. A (identical index sets in f^(0)
 * and f^(1)): index string, multiplicity printed in front of the term, and
 * the order (whose prefactor is 1/(2cs^6), 1/(4cs^8), 1/(4cs^10), 1/(8cs^12)). */
typedef struct { int n; int al[6]; double mult; } term_t;
enum { X_ = 0, Y_ = 1, Z_ = 2 };
static const term_t g_terms[] = {
    {3, {X_, X_, Y_}, 1.0}, {3, {X_, X_, Z_}, 1.0}, {3, {X_, Y_, Y_}, 1.0},
    {3, {X_, Z_, Z_}, 1.0}, {3, {Y_, Z_, Z_}, 1.0}, {3, {Y_, Y_, Z_}, 1.0},
    {3, {X_, Y_, Z_}, 2.0},
    {4, {X_, X_, Y_, Y_}, 1.0}, {4, {X_, X_, Z_, Z_}, 1.0}, {4, {Y_, Y_, Z_, Z_}, 1.0},
    {4, {X_, Y_, Z_, Z_}, 2.0}, {4, {X_, Y_, Y_, Z_}, 2.0}, {4, {X_, X_, Y_, Z_}, 2.0},
    {5, {X_, X_, Y_, Z_, Z_}, 1.0}, {5, {X_, X_, Y_, Y_, Z_}, 1.0},
    {5, {X_, Y_, Y_, Z_, Z_}, 1.0},
    {6, {X_, X_, Y_, Y_, Z_, Z_}, 1.0},
};
#define NTERMS ((int)(sizeof(g_terms) / sizeof(g_terms[0])))

static double order_prefactor(int n)
{
    switch (n) {
    case 3: return 1.0 / (2.0 * pow(CS2, 3));
    case 4: return 1.0 / (4.0 * pow(CS2, 4));
    case 5: return 1.0 / (4.0 * pow(CS2, 5));
    case 6: return 1.0 / (8.0 * pow(CS2, 6));
    }
    return 0.0;
}

static double g_H2[Q][3][3];        /* H^(2)_i,ab  */
static double g_Ht[Q][NTERMS];      /* H^(n)_i for each printed term */

/* D3Q27 velocities (Sec. 2.1; k,l,m = 0..2 read as -1,0,1) and weights.
 * The paper prints no weights; the D3Q27 weights of the cited lattice are the
 * products of the one-dimensional weights 2/3 (rest) and 1/6 (moving). */
void orc_init(void)
{
    if (g_ready) return;
    for (int i = 0; i < Q; i++) {
        g_xi[i][0] = i % 3 - 1;
        g_xi[i][1] = (i / 3) % 3 - 1;
        g_xi[i][2] = i / 9 - 1;
        double w = 1.0;
        for (int d = 0; d < 3; d++) w *= (g_xi[i][d] == 0) ? 2.0 / 3.0 : 1.0 / 6.0;
        g_w[i] = w;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                int al[2] = {a, b};
                g_H2[i][a][b] = hermite(g_xi[i], al, 2);
            }
        for (int t = 0; t < NTERMS; t++) g_Ht[i][t] = hermite(g_xi[i], g_terms[t].al, g_terms[t].n);
    }
    g_ready = 1;
}

void orc_lattice(int32_t *xi_out, double *w_out)
{
    orc_init();
    for (int i = 0; i < Q; i++) {
        for (int d = 0; d < 3; d++) xi_out[3 * i + d] = g_xi[i][d];
        w_out[i] = g_w[i];
    }
}

double orc_hermite(int32_t i, const int32_t *al, int32_t n)
{
    orc_init();
    int a[8];
    for (int k = 0; k < n; k++) a[k] = al[k];
    return hermite(g_xi[i], a, n);
}

/* ----------------------------------------------------- moments (Sec. 2.1) */

static void moments(const double *f, double *rho, double *p, double u[3])
{
    double s = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; i++) {
        s += f[i];
        for (int d = 0; d < 3; d++) j[d] += g_xi[i][d] * f[i];
    }
    *rho = s;
    *p = CS2 * (s - RHO0);
    for (int d = 0; d < 3; d++) u[d] = j[d] / s;
}

/* ---------------------------------------------- equilibrium (App. A, f^(0)) */

void orc_feq(double p, const double *u, double *out)
{
    orc_init();
    double dens = p / CS2 + RHO0;
    for (int i = 0; i < Q; i++) {
        double s = 1.0;
        double xu = 0.0;
        for (int d = 0; d < 3; d++) xu += g_xi[i][d] * u[d];
        s += xu / CS2;
        double h2 = 0.0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) h2 += g_H2[i][a][b] * u[a] * u[b];
        s += h2 / (2.0 * CS2 * CS2);
        for (int t = 0; t < NTERMS; t++) {
            double mono = 1.0;
            for (int k = 0; k < g_terms[t].n; k++) mono *= u[g_terms[t].al[k]];
            s += order_prefactor(g_terms[t].n) * g_terms[t].mult * g_Ht[i][t] * mono;
        }
        out[i] = g_w[i] * dens * s;
    }
}

/* ------------------------------ recursion for a_1^(n) (App. A, eq. rel_a1)
 * a^(n)_{a1..an} = a^(n-1)_{a1..a(n-1)} u_an
 *                 + sum over the cyclic permutations b of (a1..a(n-1)) of
 *                   u_b1 ... u_b(n-2) P^(1)_{b(n-1) an},
 * started from a^(2) = P^(1). */
static double a1_rec(const double P1[3][3], const double u[3], const int *al, int n)
{
    if (n == 2) return P1[al[0]][al[1]];
    double s = a1_rec(P1, u, al, n - 1) * u[al[n - 1]];
    int m = n - 1;
    for (int r = 0; r < m; r++) {
        double prod = 1.0;
        for (int k = 0; k < m - 1; k++) prod *= u[al[(k + r) % m]];
        s += prod * P1[al[(m - 1 + r) % m]][al[n - 1]];
    }
    return s;
}

double orc_a1(const double *P1flat, const double *u, const int32_t *al, int32_t n)
{
    double P1[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) P1[a][b] = P1flat[3 * a + b];
    int a[8];
    for (int k = 0; k < n; k++) a[k] = al[k];
    return a1_rec(P1, u, a, n);
}

/* ------------------------------------------ off-equilibrium (App. A, f^(1)) */

void orc_fneq(const double *P1flat, const double *u, double *out)
{
    orc_init();
    double P1[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) P1[a][b] = P1flat[3 * a + b];
    double a1[NTERMS];
    for (int t = 0; t < NTERMS; t++) a1[t] = a1_rec(P1, u, g_terms[t].al, g_terms[t].n);
    for (int i = 0; i < Q; i++) {
        double h2 = 0.0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) h2 += g_H2[i][a][b] * P1[a][b];
        double s = h2 / (2.0 * CS2 * CS2);
        for (int t = 0; t < NTERMS; t++)
            s += order_prefactor(g_terms[t].n) * g_terms[t].mult * g_Ht[i][t] * a1[t];
        out[i] = g_w[i] * s;
    }
}

/* P^(1) = sum_i xi_i xi_i (f_i - f^(0)_i) (App. A), with the unforced f^(0)(p,u). */
static void offeq_moment(const double *f, const double *f0, double P1[3][3])
{
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double s = 0.0;
            for (int i = 0; i < Q; i++) s += g_xi[i][a] * g_xi[i][b] * (f[i] - f0[i]);
            P1[a][b] = s;
        }
}

/* ------------------------------------------------------ collision (Sec. 2.1/2.2)
 * C_i = f^(0)_i(p, u + tau h) + (1 - 1/tau) f^(1)_i, i.e. the forced evolution
 * rule before the shift x -> x + xi_i.  Readings: f^(1) is built from P^(1) of
 * the unshifted f^(0)(p,u); u is sum xi f / sum f of the incoming f. */
/* collision = 0: the recursive-regularized rule above; collision = 1: BGK
 * for comparison, the same rule with the raw off-equilibrium f - f^(0)(p,u)
 * in place of the regularized f^(1). */
void orc_collide_cell_m(const double *f, const double *h, double tau, int32_t forcing, int32_t collision,
                        double *out)
{
    orc_init();
    double rho, p, u[3], f0[Q], f1[Q], fs[Q], P1[3][3], P1f[9], us[3];
    moments(f, &rho, &p, u);
    orc_feq(p, u, f0);
    if (collision == 1) {
        for (int i = 0; i < Q; i++) f1[i] = f[i] - f0[i];
    } else {
        offeq_moment(f, f0, P1);
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) P1f[3 * a + b] = P1[a][b];
        orc_fneq(P1f, u, f1);
    }
    for (int d = 0; d < 3; d++) us[d] = u[d] + tau * (h ? h[d] : 0.0);
    orc_feq(p, us, fs);
    for (int i = 0; i < Q; i++) out[i] = fs[i] + (1.0 - 1.0 / tau) * f1[i];
    /* Momentum-exact variant (forcing = 1): f^(0)(p, u + tau h) carries the
     * momentum rho (u + tau h) and f^(1) none, so the rule as printed adds
     * tau rho h per step.  Removing (tau - 1) rho h from the first-order
     * Hermite term, w_i (xi_i . m) / cs^2 with m = (tau - 1) rho h, leaves the
     * added momentum at rho h; mass and the second moment are unchanged
     * because sum_i w_i xi_i = 0 and sum_i w_i xi_i xi_i xi_i = 0. */
    if (forcing == 1 && h) {
        for (int i = 0; i < Q; i++) {
            double xh = g_xi[i][0] * h[0] + g_xi[i][1] * h[1] + g_xi[i][2] * h[2];
            out[i] -= g_w[i] * (tau - 1.0) * rho * xh / CS2;
        }
    }
}

void orc_collide_cell_v(const double *f, const double *h, double tau, int32_t forcing, double *out)
{
    orc_collide_cell_m(f, h, tau, forcing, 0, out);
}

void orc_collide_cell(const double *f, const double *h, double tau, double *out)
{
    orc_collide_cell_v(f, h, tau, 0, out);
}

/* --------------------------------------------------------- stress (Sec. 2.1)
 * sigma = -p I + (1/(2 tau) - 1) sum_i xi_i xi_i (f_i - f^(0)_i).
 * Also returns rho and u (the u* of Sec. 2.2). */
void orc_stress_cell(const double *f, double tau, double *sigma9, double *rho_out, double *u_out)
{
    orc_init();
    double rho, p, u[3], f0[Q], P1[3][3];
    moments(f, &rho, &p, u);
    orc_feq(p, u, f0);
    offeq_moment(f, f0, P1);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            sigma9[3 * a + b] = (a == b ? -p : 0.0) + (1.0 / (2.0 * tau) - 1.0) * P1[a][b];
    if (rho_out) *rho_out = rho;
    if (u_out)
        for (int d = 0; d < 3; d++) u_out[d] = u[d];
}

/* --------------------------------------------- weight function (Sec. 2.2) */
double orc_phi(double r)
{
    double a = fabs(r);
    if (a <= 1.0) return 0.125 * (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * r * r));
    if (a <= 2.0) return 0.125 * (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * r * r));
    return 0.0;
}

/* ------------------------------------------- storage quantization (build)
 * The precision form of the build stores each population as s_i (f_i - w_i)
 * in IEEE binary16 or in bfloat16, rounded to nearest with ties to even;
 * s_i = 2^(14 + 2 |xi_i|^2), the first power of two at or above 4096 / w_i,
 * so that scaling by it is exact.  The paper has no reduced-precision storage; this models the
 * stored state so that the GPU's reduced-precision path can be compared
 * element by element.  A value of a binary format with p significand bits
 * (the leading one included), smallest normal exponent emin and largest
 * finite value vmax is an integer multiple of 2^(E - p + 1), where E is the
 * exponent of its leading bit, clamped at emin below (subnormals); rounding
 * to that grid with nearbyint under the default rounding mode rounds ties to
 * even, and a rounded magnitude above vmax overflows to infinity. */
static double round_to_format(double x, int p, int emin, double vmax)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    (void)frexp(fabs(x), &e);          /* |x| in [2^(e-1), 2^e) */
    int E = e - 1;
    if (E < emin) E = emin;
    const double ulp = ldexp(1.0, E - (p - 1));
    const double r = nearbyint(x / ulp) * ulp;
    if (fabs(r) > vmax) return copysign(INFINITY, x);
    return r;
}

enum { STORE_F64 = 0, STORE_F16 = 1, STORE_BF16 = 2 };

double orc_round_format(double x, int32_t storage)
{
    if (storage == STORE_F16) return round_to_format(x, 11, -14, 65504.0);
    if (storage == STORE_BF16) return round_to_format(x, 8, -126, ldexp(255.0, 120));
    return x;
}

/* One population as the stored state keeps it: w_i + q(s_i (f_i - w_i)) / s_i. */
static double quantize_pop(double f, int i, int32_t storage)
{
    const int n2 = g_xi[i][0] * g_xi[i][0] + g_xi[i][1] * g_xi[i][1] + g_xi[i][2] * g_xi[i][2];
    const double s = ldexp(1.0, 14 + 2 * n2);
    return g_w[i] + orc_round_format(s * (f - g_w[i]), storage) / s;
}

/* The same on a whole field of n cells (layout cell*27 + i). */
void orc_quantize(int32_t storage, int64_t n, double *f)
{
    orc_init();
    if (storage == STORE_F64) return;
    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; c++)
        for (int i = 0; i < Q; i++) f[Q * c + i] = quantize_pop(f[Q * c + i], i, storage);
}

/* ------------------------------------------------------------- domain */

enum { BC_PERIODIC = 0, BC_FREESLIP = 1, BC_NOSLIP = 2, BC_PRESSURE = 3 };

typedef struct {
    int nx, ny, nz;
    double tau0;
    int bc_lo, bc_hi, sponge;
    int forcing;    /* 0: forced rule as printed; 1: momentum-exact variant */
    int collision;  /* 0: recursive regularized (the paper's); 1: BGK */
    double uw_lo, uw_hi;   /* x velocity of a no-slip bottom / top wall */
} dom_t;

/* Relaxation time at height z.  Sponge reading (Sec. 2.5): tau rises linearly
 * from tau0 at z_s = nz - sponge to 1 at the top row z = nz - 1. */
static double tau_at(const dom_t *D, int z)
{
    if (D->sponge < 2) return D->tau0;
    int zs = D->nz - D->sponge;
    if (z < zs) return D->tau0;
    return D->tau0 + (1.0 - D->tau0) * (double)(z - zs) / (double)(D->nz - 1 - zs);
}

double orc_tau_at(int32_t nz, double tau0, int32_t sponge, int32_t z)
{
    dom_t D = {1, 1, nz, tau0, 0, 0, sponge};
    return tau_at(&D, z);
}

static inline int wrap(int a, int n) { a %= n; return a < 0 ? a + n : a; }
static inline size_t cell(const dom_t *D, int x, int y, int z)
{
    return (size_t)x + (size_t)D->nx * ((size_t)y + (size_t)D->ny * (size_t)z);
}

/* Collision of every cell (h may be NULL = no immersed force). */
static void collide_grid(const dom_t *D, const double *f, const double *h, double *C)
{
    #pragma omp parallel for schedule(static)
    for (int z = 0; z < D->nz; z++) {
        double tau = tau_at(D, z);
        for (int y = 0; y < D->ny; y++)
            for (int x = 0; x < D->nx; x++) {
                size_t c = cell(D, x, y, z);
                orc_collide_cell_m(f + Q * c, h ? h + 3 * c : NULL, tau, D->forcing, D->collision, C + Q * c);
            }
    }
}

/* Streaming f_i(x) = C_i(x - xi_i) (Sec. 2.1 evolution rule, pull form).
 * Lateral walls periodic (Sec. 2.5).  z walls at z = -1/2 and nz - 1/2:
 * periodic, free-slip (specular reflection, xi_z flipped), no-slip
 * (bounce-back, whole xi reversed) or constant pressure (the Sec. 3 domain
 * top, density rho0 = 1 at the halfway plane; reading: anti-bounce-back
 * f_i = -C_opp(i) + 2 w_i rho0, the O(u^2) wall-velocity terms dropped).
 * A no-slip wall moving in x at u_w (the shear flow of the rotation case):
 * bounce-back plus the wall's momentum, f_i = C_opp(i) + 2 w_i rho0 xi_i.u_w / cs^2. */
static void stream_grid(const dom_t *D, const double *C, double *f)
{
    #pragma omp parallel for schedule(static)
    for (int z = 0; z < D->nz; z++)
        for (int y = 0; y < D->ny; y++)
            for (int x = 0; x < D->nx; x++) {
                size_t c = cell(D, x, y, z);
                for (int i = 0; i < Q; i++) {
                    int sx = wrap(x - g_xi[i][0], D->nx);
                    int sy = wrap(y - g_xi[i][1], D->ny);
                    int sz = z - g_xi[i][2];
                    int bc = sz < 0 ? D->bc_lo : (sz >= D->nz ? D->bc_hi : -1);
                    if (bc == -1) {
                        f[Q * c + i] = C[Q * cell(D, sx, sy, sz) + i];
                    } else if (bc == BC_PERIODIC) {
                        f[Q * c + i] = C[Q * cell(D, sx, sy, wrap(sz, D->nz)) + i];
                    } else if (bc == BC_FREESLIP) {
                        int im = 9 * (-g_xi[i][2] + 1) + 3 * (g_xi[i][1] + 1) + (g_xi[i][0] + 1);
                        f[Q * c + i] = C[Q * cell(D, sx, sy, z) + im];
                    } else if (bc == BC_PRESSURE) {
                        f[Q * c + i] = -C[Q * c + (Q - 1 - i)] + 2.0 * g_w[i] * RHO0;
                    } else {
                        const double uw = sz < 0 ? D->uw_lo : D->uw_hi;
                        f[Q * c + i] = C[Q * c + (Q - 1 - i)] + 2.0 * g_w[i] * RHO0 * g_xi[i][0] * uw / CS2;
                    }
                }
            }
}

void orc_collide_grid_m(const int32_t *dims, double tau0, int32_t sponge, int32_t forcing, int32_t collision,
                        const double *f, const double *h, double *C)
{
    orc_init();
    dom_t D = {dims[0], dims[1], dims[2], tau0, 0, 0, sponge, forcing, collision};
    collide_grid(&D, f, h, C);
}

void orc_collide_grid_v(const int32_t *dims, double tau0, int32_t sponge, int32_t forcing, const double *f,
                        const double *h, double *C)
{
    orc_collide_grid_m(dims, tau0, sponge, forcing, 0, f, h, C);
}

void orc_collide_grid(const int32_t *dims, double tau0, int32_t sponge, const double *f,
                      const double *h, double *C)
{
    orc_collide_grid_v(dims, tau0, sponge, 0, f, h, C);
}

void orc_stream_grid(const int32_t *dims, int32_t bc_lo, int32_t bc_hi, const double *C, double *f)
{
    orc_init();
    dom_t D = {dims[0], dims[1], dims[2], 1.0, bc_lo, bc_hi, 0};
    stream_grid(&D, C, f);
}

/* The same with no-slip walls moving in x at uw[0] (bottom) and uw[1] (top). */
void orc_stream_grid_w(const int32_t *dims, int32_t bc_lo, int32_t bc_hi, const double *uw, const double *C, double *f)
{
    orc_init();
    dom_t D = {dims[0], dims[1], dims[2], 1.0, bc_lo, bc_hi, 0};
    D.uw_lo = uw[0];
    D.uw_hi = uw[1];
    stream_grid(&D, C, f);
}

/* -------------------------------------------- interpolation and spreading
 * Stencil: nodes floor(X)-1 .. floor(X)+2 on each axis (w vanishes beyond),
 * periodic in x and y; nodes outside 0..nz-1 in z are an error (-1). */
static int stencil(const dom_t *D, const double X[3], int node[3][4], double wt[3][4])
{
    for (int d = 0; d < 3; d++) {
        int b = (int)floor(X[d]) - 1;
        int n = d == 0 ? D->nx : (d == 1 ? D->ny : D->nz);
        for (int a = 0; a < 4; a++) {
            int j = b + a;
            wt[d][a] = orc_phi((double)j - X[d]);
            if (d < 2) j = wrap(j, n);
            else if (j < 0 || j >= n) return -1;
            node[d][a] = j;
        }
    }
    return 0;
}

/* I[field](X) = sum_x field(x) W(x - X) dx^3, ncomp components per cell. */
static int interp(const dom_t *D, const double *field, int ncomp, const double X[3], double *out)
{
    int node[3][4];
    double wt[3][4];
    if (stencil(D, X, node, wt)) return -1;
    for (int c = 0; c < ncomp; c++) out[c] = 0.0;
    for (int c3 = 0; c3 < 4; c3++)
        for (int b = 0; b < 4; b++)
            for (int a = 0; a < 4; a++) {
                double W = wt[0][a] * wt[1][b] * wt[2][c3];
                size_t cc = cell(D, node[0][a], node[1][b], node[2][c3]);
                for (int c = 0; c < ncomp; c++) out[c] += field[ncomp * cc + c] * W;
            }
    return 0;
}

/* S[h](x) += sum_k h_k W(x - X_k) dS_k (dx = 1, so W carries no 1/dx^3). */
static int spread_add(const dom_t *D, const double X[3], const double h[3], double dS, double *H)
{
    int node[3][4];
    double wt[3][4];
    if (stencil(D, X, node, wt)) return -1;
    for (int c3 = 0; c3 < 4; c3++)
        for (int b = 0; b < 4; b++)
            for (int a = 0; a < 4; a++) {
                double W = wt[0][a] * wt[1][b] * wt[2][c3];
                size_t cc = cell(D, node[0][a], node[1][b], node[2][c3]);
                for (int d = 0; d < 3; d++) H[3 * cc + d] += h[d] * W * dS;
            }
    return 0;
}

int32_t orc_interp(const int32_t *dims, const double *field, int32_t ncomp, int32_t M,
                   const double *X, double *out)
{
    dom_t D = {dims[0], dims[1], dims[2], 1.0, 0, 0, 0};
    for (int k = 0; k < M; k++)
        if (interp(&D, field, ncomp, X + 3 * k, out + ncomp * k)) return -1;
    return 0;
}

int32_t orc_spread(const int32_t *dims, int32_t M, const double *X, const double *h,
                   const double *dS, double *H)
{
    dom_t D = {dims[0], dims[1], dims[2], 1.0, 0, 0, 0};
    size_t n = (size_t)D.nx * D.ny * D.nz;
    memset(H, 0, 3 * n * sizeof(double));
    for (int k = 0; k < M; k++)
        if (spread_add(&D, X + 3 * k, h + 3 * k, dS[k], H)) return -1;
    return 0;
}

/* ------------------------------------------------------- 3x3 helpers */

static void cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static int inv3(const double A[9], double B[9])
{
    double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                 A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (det == 0.0) return -1;
    B[0] = (A[4] * A[8] - A[5] * A[7]) / det;
    B[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    B[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    B[3] = (A[5] * A[6] - A[3] * A[8]) / det;
    B[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    B[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    B[6] = (A[3] * A[7] - A[4] * A[6]) / det;
    B[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    B[8] = (A[0] * A[4] - A[1] * A[3]) / det;
    return 0;
}

static void matvec(const double A[9], const double x[3], double y[3])
{
    for (int a = 0; a < 3; a++) y[a] = A[3 * a] * x[0] + A[3 * a + 1] * x[1] + A[3 * a + 2] * x[2];
}

/* --------------------------------------------------- rigid body (Sec. 2.3)
 * State: r, rows d_0..d_2 of the matrix M, v(t-1/2), w(t-1/2).
 *   a      = g + F / (kappa V)
 *   v     += a;           r += v
 *   w     += M^-1 (J/m)^-1 M (T + T_ext) / (kappa V)   (T_ext: constant external torque)
 *   d_pred = d + w x d;   d += w x (d + d_pred)/2
 * M^-1 is the true inverse (the paper writes M^-1; the d_i are not
 * re-orthonormalised).  Gravity g = (0, 0, -gravity). */
typedef struct {
    double r[3], d[9], v[3], w[3];
    double kappa, vol, Jm[9], gravity;
    double Text[3];
} body_t;

static void body_advance(body_t *B, const double F[3], const double T[3])
{
    double kv = B->kappa * B->vol;
    double a[3] = {F[0] / kv, F[1] / kv, F[2] / kv - B->gravity};
    for (int d = 0; d < 3; d++) {
        B->v[d] += a[d];
        B->r[d] += B->v[d];
    }
    double Minv[9], Jinv[9], t1[3], t2[3], t3[3];
    inv3(B->d, Minv);
    inv3(B->Jm, Jinv);
    const double Ttot[3] = {T[0] + B->Text[0], T[1] + B->Text[1], T[2] + B->Text[2]};
    matvec(B->d, Ttot, t1);
    matvec(Jinv, t1, t2);
    matvec(Minv, t2, t3);
    for (int d = 0; d < 3; d++) B->w[d] += t3[d] / kv;
    for (int i = 0; i < 3; i++) {
        double *di = B->d + 3 * i, dp[3], wd[3], mid[3], wm[3];
        cross(B->w, di, wd);
        for (int d = 0; d < 3; d++) dp[d] = di[d] + wd[d];
        for (int d = 0; d < 3; d++) mid[d] = 0.5 * (di[d] + dp[d]);
        cross(B->w, mid, wm);
        for (int d = 0; d < 3; d++) di[d] += wm[d];
    }
}

/* state[24] = r(3) d(9) v(3) w(3) | F(3) T(3) in;  params[12] = kappa vol Jm(9) gravity */
void orc_body_advance(double *state, const double *FT, const double *params)
{
    body_t B;
    memset(&B, 0, sizeof B);   /* FT holds the whole torque: no external part */
    memcpy(B.r, state, 3 * sizeof(double));
    memcpy(B.d, state + 3, 9 * sizeof(double));
    memcpy(B.v, state + 12, 3 * sizeof(double));
    memcpy(B.w, state + 15, 3 * sizeof(double));
    B.kappa = params[0];
    B.vol = params[1];
    memcpy(B.Jm, params + 2, 9 * sizeof(double));
    B.gravity = params[11];
    body_advance(&B, FT, FT + 3);
    memcpy(state, B.r, 3 * sizeof(double));
    memcpy(state + 3, B.d, 9 * sizeof(double));
    memcpy(state + 12, B.v, 3 * sizeof(double));
    memcpy(state + 15, B.w, 3 * sizeof(double));
}

/* ------------------------------------------------------- full simulation */

typedef struct {
    dom_t D;
    double h_ini, h_end;
    int cycles;
    int M;
    double *xb, *nb, *dS;          /* body-frame markers (M x 3), areas (M) */
    body_t B;
    double F[3], T[3], Fp[3];      /* F(t), T(t) and the pressure part of F */
    double resid;                  /* max_k |U_k - I[u* + H](X_k)| after the last spread */
    double *f, *h, *C;             /* populations, immersed force, scratch */
    double *sig, *uu;              /* stress (9) + p (1), and u* (3), at flagged nodes */
    unsigned char *need;           /* nodes covered by a marker stencil */
    double *X, *N, *U, *hk, *tmp;  /* markers at t+1 */
    int pending;                   /* window shift to apply to the next post-collision state */
    double force_offset;           /* 0: stress integral at the markers; > 0: on the parallel
                                      surface X_k + force_offset n_k, areas dSo */
    double *dSo;
    double gf[3];                  /* uniform fluid force added to h_imm in the collision */
    int storage;                   /* STORE_*: precision of the stored post-collision state */
    double box_rb;                 /* full-precision box around the body: reach and edges */
    int box_edge[3];
    double *htot;                  /* h_imm + gf when gf is set */
    int64_t shifts, steps;
    int err;
} orc_sim;

/* dims[3]; ip[6] = bc_lo bc_hi sponge cycles forcing collision; dp[4] = tau0 gravity h_ini h_end;
 * body[29] = kappa vol Jm(9) r(3) d(9) v(3) w(3). */
orc_sim *orc_sim_new(const int32_t *dims, const int32_t *ip, const double *dp, int32_t M,
                     const double *xb, const double *nb, const double *dS, const double *body)
{
    orc_init();
    orc_sim *S = (orc_sim *)calloc(1, sizeof(orc_sim));
    S->D.nx = dims[0];
    S->D.ny = dims[1];
    S->D.nz = dims[2];
    S->D.bc_lo = ip[0];
    S->D.bc_hi = ip[1];
    S->D.sponge = ip[2];
    S->D.forcing = ip[4];
    S->D.collision = ip[5];
    S->cycles = ip[3];
    S->D.tau0 = dp[0];
    S->B.gravity = dp[1];
    S->h_ini = dp[2];
    S->h_end = dp[3];
    S->M = M;
    size_t n = (size_t)S->D.nx * S->D.ny * S->D.nz;
    S->f = (double *)malloc(Q * n * sizeof(double));
    S->C = (double *)malloc(Q * n * sizeof(double));
    S->h = (double *)calloc(3 * n, sizeof(double));
    S->sig = (double *)calloc(10 * n, sizeof(double));
    S->uu = (double *)calloc(3 * n, sizeof(double));
    S->need = (unsigned char *)calloc(n, 1);
    int mm = M > 0 ? M : 1;
    S->xb = (double *)malloc(3 * mm * sizeof(double));
    S->nb = (double *)malloc(3 * mm * sizeof(double));
    S->dS = (double *)malloc(mm * sizeof(double));
    S->X = (double *)malloc(3 * mm * sizeof(double));
    S->N = (double *)malloc(3 * mm * sizeof(double));
    S->U = (double *)malloc(3 * mm * sizeof(double));
    S->hk = (double *)malloc(3 * mm * sizeof(double));
    S->tmp = (double *)malloc(10 * mm * sizeof(double));
    if (M > 0) {
        memcpy(S->xb, xb, 3 * M * sizeof(double));
        memcpy(S->nb, nb, 3 * M * sizeof(double));
        memcpy(S->dS, dS, M * sizeof(double));
    }
    S->B.kappa = body[0];
    S->B.vol = body[1];
    memcpy(S->B.Jm, body + 2, 9 * sizeof(double));
    memcpy(S->B.r, body + 11, 3 * sizeof(double));
    memcpy(S->B.d, body + 14, 9 * sizeof(double));
    memcpy(S->B.v, body + 23, 3 * sizeof(double));
    memcpy(S->B.w, body + 26, 3 * sizeof(double));
    /* initial state (Table 1 (0)): fluid at rest f = w, h = 0, F = T = 0 */
    for (size_t c = 0; c < n; c++)
        for (int i = 0; i < Q; i++) S->f[Q * c + i] = g_w[i];
    return S;
}

/* Force surface variant: the stress integral on the parallel surface at
 * distance delta outside the markers, with its marker areas dSo (M values). */
/* Constant external torque (lab frame) added to the fluid torque in the
 * angular update (App. B spins a sphere up from rest this way). */
void orc_sim_set_torque(orc_sim *S, const double *T)
{
    for (int a = 0; a < 3; a++) S->B.Text[a] = T[a];
}

/* x velocities of the bottom and top walls (no-slip walls only). */
void orc_sim_set_walls(orc_sim *S, const double *uw)
{
    S->D.uw_lo = uw[0];
    S->D.uw_hi = uw[1];
}

void orc_sim_set_force_surface(orc_sim *S, double delta, const double *dSo)
{
    S->force_offset = delta;
    free(S->dSo);
    S->dSo = NULL;
    if (delta > 0.0 && S->M > 0) {
        S->dSo = (double *)malloc(S->M * sizeof(double));
        memcpy(S->dSo, dSo, S->M * sizeof(double));
    }
}

/* A uniform force per unit mass on the fluid (a mean pressure gradient in a
 * periodic box).  It enters the forced rule of Sec. 2.2 exactly like the
 * immersed force: the collision evaluates f^(0) at u + tau (h_imm + gf). */
void orc_sim_set_fluid_force(orc_sim *S, const double *gf)
{
    size_t n = (size_t)S->D.nx * S->D.ny * S->D.nz;
    for (int a = 0; a < 3; a++) S->gf[a] = gf[a];
    if (!S->htot) S->htot = (double *)malloc(3 * n * sizeof(double));
}

/* Reduced-precision storage of the post-collision state (the build's
 * precision form): after each collision every population is replaced by the
 * value the stored format holds.  With box edges > 0 the cells of a box
 * around the body keep full precision: per axis a the cells
 * floor(r_a - box_rb) - 3 ... + box_edge[a] - 1 (x and y periodic, z not
 * wrapped), r being the body position of the stored state. */
void orc_sim_set_storage(orc_sim *S, int32_t storage, double box_rb, const int32_t *box_edge)
{
    S->storage = storage;
    S->box_rb = box_rb;
    for (int a = 0; a < 3; a++) S->box_edge[a] = box_edge ? box_edge[a] : 0;
}

static void quantize_state(orc_sim *S, double *C)
{
    if (S->storage == STORE_F64) return;
    const dom_t *D = &S->D;
    int lo[3] = {0, 0, 0};
    const int *e = S->box_edge;
    const int boxed = e[0] > 0 && e[1] > 0 && e[2] > 0;
    if (boxed) {
        /* a window shift still pending moves this state up later: its body
         * position is r_z - pending until then */
        const double r[3] = {S->B.r[0], S->B.r[1], S->B.r[2] - S->pending};
        for (int a = 0; a < 3; a++) lo[a] = (int)floor(r[a] - S->box_rb) - 3;
    }
    #pragma omp parallel for schedule(static)
    for (int z = 0; z < D->nz; z++)
        for (int y = 0; y < D->ny; y++)
            for (int x = 0; x < D->nx; x++) {
                if (boxed) {
                    const int kx = wrap(x - lo[0], D->nx), ky = wrap(y - lo[1], D->ny), kz = z - lo[2];
                    if (kx < e[0] && ky < e[1] && kz >= 0 && kz < e[2]) continue;
                }
                const size_t c = cell(D, x, y, z);
                for (int i = 0; i < Q; i++) C[Q * c + i] = quantize_pop(C[Q * c + i], i, S->storage);
            }
}

void orc_sim_free(orc_sim *S)
{
    if (!S) return;
    free(S->f); free(S->C); free(S->h); free(S->sig); free(S->uu); free(S->need);
    free(S->xb); free(S->nb); free(S->dS); free(S->X); free(S->N); free(S->U);
    free(S->hk); free(S->tmp); free(S->dSo); free(S->htot);
    free(S);
}

/* The force field the collision applies: h_imm, plus the uniform fluid force
 * when one is set. */
static const double *forcing_field(orc_sim *S)
{
    if (!S->htot) return S->h;
    size_t n = (size_t)S->D.nx * S->D.ny * S->D.nz;
    for (size_t c = 0; c < n; c++)
        for (int a = 0; a < 3; a++) S->htot[3 * c + a] = S->h[3 * c + a] + S->gf[a];
    return S->htot;
}

void orc_sim_set_f(orc_sim *S, const double *f)
{
    size_t n = (size_t)S->D.nx * S->D.ny * S->D.nz;
    memcpy(S->f, f, Q * n * sizeof(double));
}

void orc_sim_get_f(const orc_sim *S, double *f)
{
    size_t n = (size_t)S->D.nx * S->D.ny * S->D.nz;
    memcpy(f, S->f, Q * n * sizeof(double));
}

void orc_sim_get_h(const orc_sim *S, double *h)
{
    size_t n = (size_t)S->D.nx * S->D.ny * S->D.nz;
    memcpy(h, S->h, 3 * n * sizeof(double));
}

/* Falling-frame re-injection (Sec. 2.5).  Reading: the whole window content
 * moves up by an integer Delta = round(h_ini - h_end) cells; the top Delta
 * slabs leave the window, the bottom Delta slabs restart at rest (f = w),
 * and the particle moves up by Delta.  The copy acts on the post-collision
 * populations of the following step. */
static void shift_post_collision(orc_sim *S, double *C)
{
    const dom_t *D = &S->D;
    int dz = S->pending;
    size_t slab = (size_t)D->nx * D->ny;
    for (int z = D->nz - 1; z >= 0; z--) {
        double *dst = C + Q * slab * (size_t)z;
        if (z >= dz) {
            memcpy(dst, C + Q * slab * (size_t)(z - dz), Q * slab * sizeof(double));
        } else {
            for (size_t c = 0; c < slab; c++)
                for (int i = 0; i < Q; i++) dst[Q * c + i] = g_w[i];
        }
    }
    S->pending = 0;
}

/* Post-collision populations C_t = collide(f(t), h(t)) (with a pending
 * window shift applied), i.e. the state a pull-scheme solver keeps between
 * steps. */
void orc_sim_get_post_collision(orc_sim *S, double *C)
{
    collide_grid(&S->D, S->f, forcing_field(S), C);
    quantize_state(S, C);
    if (S->pending) {
        int keep = S->pending;
        shift_post_collision(S, C);
        S->pending = keep;
    }
}

/* Markers at the current body state (Sec. 2.3):
 *   X_k = r + sum_j xb_kj d_j,  n_k = sum_j nb_kj d_j,  U_k = v + w x (X_k - r). */
static void place_markers(orc_sim *S)
{
    for (int k = 0; k < S->M; k++) {
        for (int a = 0; a < 3; a++) {
            double xs = S->B.r[a], ns = 0.0;
            for (int j = 0; j < 3; j++) {
                xs += S->xb[3 * k + j] * S->B.d[3 * j + a];
                ns += S->nb[3 * k + j] * S->B.d[3 * j + a];
            }
            S->X[3 * k + a] = xs;
            S->N[3 * k + a] = ns;
        }
        double rel[3], wr[3];
        for (int a = 0; a < 3; a++) rel[a] = S->X[3 * k + a] - S->B.r[a];
        cross(S->B.w, rel, wr);
        for (int a = 0; a < 3; a++) S->U[3 * k + a] = S->B.v[a] + wr[a];
    }
}

/* Stress and u* at every node that some marker stencil touches (the only
 * nodes the interpolations read). */
static void stress_at_stencils(orc_sim *S)
{
    const dom_t *D = &S->D;
    size_t n = (size_t)D->nx * D->ny * D->nz;
    memset(S->need, 0, n);
    for (int k = 0; k < S->M; k++) {
        int node[3][4];
        double wt[3][4];
        if (stencil(D, S->X + 3 * k, node, wt)) { S->err = -1; return; }
        for (int c = 0; c < 4; c++)
            for (int b = 0; b < 4; b++)
                for (int a = 0; a < 4; a++) S->need[cell(D, node[0][a], node[1][b], node[2][c])] = 1;
        if (S->force_offset > 0.0) {
            double Y[3];
            for (int a = 0; a < 3; a++) Y[a] = S->X[3 * k + a] + S->force_offset * S->N[3 * k + a];
            if (stencil(D, Y, node, wt)) { S->err = -1; return; }
            for (int c = 0; c < 4; c++)
                for (int b = 0; b < 4; b++)
                    for (int a = 0; a < 4; a++) S->need[cell(D, node[0][a], node[1][b], node[2][c])] = 1;
        }
    }
    #pragma omp parallel for schedule(static)
    for (int z = 0; z < D->nz; z++)
        for (int y = 0; y < D->ny; y++)
            for (int x = 0; x < D->nx; x++) {
                size_t c = cell(D, x, y, z);
                if (!S->need[c]) continue;
                double rho;
                orc_stress_cell(S->f + Q * c, tau_at(D, z), S->sig + 10 * c, &rho, S->uu + 3 * c);
                S->sig[10 * c + 9] = CS2 * (rho - RHO0);
            }
}

/* Force and torque from the stress integral (Sec. 2.2), summed over the
 * markers in index order.  Torque reading: T = sum dS (X_k - C_m) x (sigma n),
 * the moment of the surface traction about the centre of mass C_m = r. */
static void force_torque(orc_sim *S)
{
    double F[3] = {0, 0, 0}, T[3] = {0, 0, 0}, Fp[3] = {0, 0, 0};
    for (int k = 0; k < S->M; k++) {
        double sg[10], s[3], rel[3], rs[3], Y[3];
        const double *nk = S->N + 3 * k;
        /* evaluation point: the marker, or its image on the parallel surface
         * at distance force_offset along the outward normal (same normal) */
        for (int a = 0; a < 3; a++) Y[a] = S->X[3 * k + a] + S->force_offset * nk[a];
        const double area = S->force_offset > 0.0 ? S->dSo[k] : S->dS[k];
        interp(&S->D, S->sig, 10, Y, sg);
        for (int a = 0; a < 3; a++) s[a] = sg[3 * a] * nk[0] + sg[3 * a + 1] * nk[1] + sg[3 * a + 2] * nk[2];
        double p = sg[9];   /* interpolated pressure: the -pI part of sigma */
        for (int a = 0; a < 3; a++) rel[a] = Y[a] - S->B.r[a];
        cross(rel, s, rs);
        for (int a = 0; a < 3; a++) {
            F[a] += area * s[a];
            T[a] += area * rs[a];
            Fp[a] += area * (-p) * nk[a];
        }
    }
    memcpy(S->F, F, sizeof F);
    memcpy(S->T, T, sizeof T);
    memcpy(S->Fp, Fp, sizeof Fp);
}

/* Multi-direct forcing (Sec. 2.2): n cycles of steps l = 0..4; the immersed
 * force is the spread of the last cycle.  Only nodes touched by the markers
 * carry a nonzero h_imm. */
static void ibm(orc_sim *S)
{
    const dom_t *D = &S->D;
    size_t n = (size_t)D->nx * D->ny * D->nz;
    int M = S->M;
    double *I = S->tmp;
    /* l = 0: h_k = (U_k - u*(X_k)) / dt */
    for (int k = 0; k < M; k++) {
        interp(D, S->uu, 3, S->X + 3 * k, I + 3 * k);
        for (int a = 0; a < 3; a++) S->hk[3 * k + a] = S->U[3 * k + a] - I[3 * k + a];
    }
    double *u2 = (double *)malloc(3 * n * sizeof(double));
    for (int c = 1; c <= S->cycles; c++) {
        /* l = 1: h_imm(x) = sum_k h_k W(x - X_k) dS_k */
        memset(S->h, 0, 3 * n * sizeof(double));
        for (int k = 0; k < M; k++) spread_add(D, S->X + 3 * k, S->hk + 3 * k, S->dS[k], S->h);
        /* l = 2: u_2 = u* + h_imm dt (at the nodes the markers read) */
        for (size_t q = 0; q < n; q++)
            if (S->need[q])
                for (int a = 0; a < 3; a++) u2[3 * q + a] = S->uu[3 * q + a] + S->h[3 * q + a];
        /* l = 3: u_3(X_k) = I[u_2](X_k) */
        double res = 0.0;
        for (int k = 0; k < M; k++) {
            interp(D, u2, 3, S->X + 3 * k, I + 3 * k);
            for (int a = 0; a < 3; a++) {
                double e = fabs(S->U[3 * k + a] - I[3 * k + a]);
                if (e > res) res = e;
            }
        }
        S->resid = res;
        if (c == S->cycles) break;   /* the last cycle's l = 1 is h_imm */
        /* l = 4: h_k += (U_k - u_3(X_k)) / dt */
        for (int k = 0; k < M; k++)
            for (int a = 0; a < 3; a++) S->hk[3 * k + a] += S->U[3 * k + a] - I[3 * k + a];
    }
    free(u2);
}

/* One time iteration in the order of Table 1:
 *   (1) collide with f(t), h(t), then stream -> f(t+1)
 *   (2) advance the particle with F(t), T(t)   -> r, d(t+1), v, w(t+1/2)
 *   (3) stress from f(t+1); F(t+1), T(t+1) at the markers X(t+1)
 *   (4) IBM iterations                        -> h(t+1)
 * then the falling-frame test of Sec. 2.5. */
int32_t orc_sim_step(orc_sim *S, int32_t nsteps)
{
    for (int s = 0; s < nsteps; s++) {
        collide_grid(&S->D, S->f, forcing_field(S), S->C);
        quantize_state(S, S->C);
        if (S->pending) shift_post_collision(S, S->C);
        stream_grid(&S->D, S->C, S->f);
        body_advance(&S->B, S->F, S->T);
        if (S->M > 0) {
            place_markers(S);
            stress_at_stencils(S);
            if (S->err) return S->err;
            force_torque(S);
            ibm(S);
        }
        S->steps++;
        if (S->h_end > 0.0 && S->B.r[2] < S->h_end) {
            int dz = (int)lround(S->h_ini - S->h_end);
            if (dz > 0) {
                S->B.r[2] += dz;
                S->pending = dz;
                S->shifts++;
            }
        }
    }
    return 0;
}

/* out[34] = r(3) d(9) v(3) w(3) F(3) T(3) Fp(3) resid steps shifts pending + 4 spare */
void orc_sim_get_body(const orc_sim *S, double *out)
{
    memcpy(out, S->B.r, 3 * sizeof(double));
    memcpy(out + 3, S->B.d, 9 * sizeof(double));
    memcpy(out + 12, S->B.v, 3 * sizeof(double));
    memcpy(out + 15, S->B.w, 3 * sizeof(double));
    memcpy(out + 18, S->F, 3 * sizeof(double));
    memcpy(out + 21, S->T, 3 * sizeof(double));
    memcpy(out + 24, S->Fp, 3 * sizeof(double));
    out[27] = S->resid;
    out[28] = (double)S->steps;
    out[29] = (double)S->shifts;
    out[30] = (double)S->pending;
}

/* Markers at the last step (X, n, U, h_k), each M x 3. */
void orc_sim_get_markers(const orc_sim *S, double *X, double *N, double *U, double *hk)
{
    size_t b = 3 * (size_t)S->M * sizeof(double);
    if (X) memcpy(X, S->X, b);
    if (N) memcpy(N, S->N, b);
    if (U) memcpy(U, S->U, b);
    if (hk) memcpy(hk, S->hk, b);
}

/* Threads of the OpenMP loops (for timing the oracle on one core). */
void orc_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int32_t orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
