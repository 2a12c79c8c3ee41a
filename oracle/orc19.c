/* orc19.c -- FP64 reference of the fluid step on the D3Q19 lattice, the
 * lattice the paper sets its D3Q27 choice against for stability (Sec. 2.1).
 *
 * TEST INFRASTRUCTURE ONLY: linked into the oracle library beside orc.c,
 * called by the tests; the product path never loads it.
 *
 * Velocities: the 19 vectors of {-1, 0, 1}^3 with |xi|^2 <= 2, ordered by
 * the D3Q27 index 9 (xi_z + 1) + 3 (xi_y + 1) + (xi_x + 1) with the eight
 * corners left out.  Weights 1/3 (rest), 1/18 (faces), 1/36 (edges); cs^2 = 1/3.
 *
 * Collision models: the construction of the D3Q27 model of App. A on the
 * Hermite polynomials D3Q19 carries.  Orders 0..2 in full.  At third order
 * the xxx and xyz types vanish on these velocities, and the six others are
 * not orthogonal on them in pairs (H_xxy with H_yzz, H_xzz with H_xyy,
 * H_yyz with H_xxz): each pair enters through its sum S and difference D,
 * which are orthogonal, with their lattice norms |S|^2 = 2 cs^6 and
 * |D|^2 = 6 cs^6, so that the moments on S and D are exact.  No fourth
 * order (on D3Q19 those polynomials are not orthogonal to the second-order
 * ones).  With a_m the continuous Hermite coefficient of a multi-index m:
 *   f0 = w [rho + xi.j / cs^2 + H2 : rho uu / (2 cs^4) + T3(a0)],  a0_m = rho u^m
 *   T3(a) = sum_pairs (a_1 + a_2) S / (2 cs^6) + (a_1 - a_2) D / (6 cs^6)
 *   P1 = sum_i xi xi (f_i - f0_i)
 *   a1^(3)_abc = P1_ab u_c + u_a P1_bc + u_b P1_ac      (the recursion of App. A at n = 3)
 *   f1 = w [H2 : P1 / (2 cs^4) + T3(a1^(3))]
 *   recursive regularized: C = f0 + (1 - 1/tau) f1;  BGK: C = f - (f - f0) / tau
 * Streaming: pull, C_i(x - xi_i), periodic in x, y and z. */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q19 19
static const double CS2_19 = 1.0 / 3.0;
static int xi19[Q19][3];
static double w19[Q19];
static int init19 = 0;

static void orc19_init(void)
{
    if (init19) return;
    int j = 0;
    for (int z = -1; z <= 1; z++)
        for (int y = -1; y <= 1; y++)
            for (int x = -1; x <= 1; x++) {
                const int n = x * x + y * y + z * z;
                if (n == 3) continue;
                xi19[j][0] = x;
                xi19[j][1] = y;
                xi19[j][2] = z;
                w19[j] = n == 0 ? 1.0 / 3.0 : (n == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
                j++;
            }
    init19 = 1;
}

void orc19_lattice(int32_t *xi, double *w)
{
    orc19_init();
    for (int i = 0; i < Q19; i++) {
        for (int a = 0; a < 3; a++) xi[3 * i + a] = xi19[i][a];
        w[i] = w19[i];
    }
}

/* Hermite tensors of order 2 and 3 at velocity i. */
static double h2(int i, int a, int b)
{
    return xi19[i][a] * xi19[i][b] - (a == b ? CS2_19 : 0.0);
}

static double h3(int i, int a, int b, int c)
{
    return (double)xi19[i][a] * xi19[i][b] * xi19[i][c] -
           CS2_19 * (xi19[i][a] * (b == c) + xi19[i][b] * (a == c) + xi19[i][c] * (a == b));
}

/* The three non-orthogonal third-order pairs: (a, a, b) with (b, c, c),
 * i.e. xxy-yzz, yyz-xxz and zzx-xyy as index triples. */
static const int PAIR[3][2][3] = {{{0, 0, 1}, {1, 2, 2}}, {{1, 1, 2}, {2, 0, 0}}, {{2, 2, 0}, {0, 1, 1}}};

/* T3(a) at velocity i for the coefficient tensor a[3][3][3]. */
static double third(int i, const double a[3][3][3])
{
    const double c6 = CS2_19 * CS2_19 * CS2_19;
    double s = 0.0;
    for (int p = 0; p < 3; p++) {
        const int *m1 = PAIR[p][0], *m2 = PAIR[p][1];
        const double h1 = h3(i, m1[0], m1[1], m1[2]), hb = h3(i, m2[0], m2[1], m2[2]);
        const double a1 = a[m1[0]][m1[1]][m1[2]], a2 = a[m2[0]][m2[1]][m2[2]];
        s += (a1 + a2) * (h1 + hb) / (2.0 * c6) + (a1 - a2) * (h1 - hb) / (6.0 * c6);
    }
    return s;
}

void orc19_feq(double rho, const double *u, double *out)
{
    orc19_init();
    double a3[3][3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            for (int c = 0; c < 3; c++) a3[a][b][c] = rho * u[a] * u[b] * u[c];
    for (int i = 0; i < Q19; i++) {
        double s1 = 0.0, s2 = 0.0;
        for (int a = 0; a < 3; a++) {
            s1 += xi19[i][a] * u[a];
            for (int b = 0; b < 3; b++) s2 += h2(i, a, b) * u[a] * u[b];
        }
        out[i] = w19[i] * (rho * (1.0 + s1 / CS2_19 + s2 / (2.0 * CS2_19 * CS2_19)) + third(i, a3));
    }
}

/* f1 of the recursive regularized model from P1 and u. */
void orc19_f1(const double *P1, const double *u, double *out)
{
    orc19_init();
    double a3[3][3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            for (int c = 0; c < 3; c++)
                a3[a][b][c] = P1[3 * a + b] * u[c] + u[a] * P1[3 * b + c] + u[b] * P1[3 * a + c];
    for (int i = 0; i < Q19; i++) {
        double s2 = 0.0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) s2 += h2(i, a, b) * P1[3 * a + b];
        out[i] = w19[i] * (s2 / (2.0 * CS2_19 * CS2_19) + third(i, a3));
    }
}

/* Post-collision populations of one cell; collision 0 = recursive
 * regularized, 1 = BGK. */
void orc19_collide_cell(const double *f, double tau, int32_t collision, double *out)
{
    orc19_init();
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q19; i++) {
        rho += f[i];
        for (int a = 0; a < 3; a++) j[a] += xi19[i][a] * f[i];
    }
    const double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    double f0[Q19];
    orc19_feq(rho, u, f0);
    if (collision == 1) {
        for (int i = 0; i < Q19; i++) out[i] = f[i] - (f[i] - f0[i]) / tau;
        return;
    }
    double P1[9];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double s = 0.0;
            for (int i = 0; i < Q19; i++) s += xi19[i][a] * xi19[i][b] * (f[i] - f0[i]);
            P1[3 * a + b] = s;
        }
    double f1[Q19];
    orc19_f1(P1, u, f1);
    for (int i = 0; i < Q19; i++) out[i] = f0[i] + (1.0 - 1.0 / tau) * f1[i];
}

static int wrap19(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

/* Collision alone on every cell of an nx x ny x nz grid, f in place. */
void orc19_collide_grid(int32_t nx, int32_t ny, int32_t nz, double tau, int32_t collision, double *f)
{
    orc19_init();
    const long long n = (long long)nx * ny * nz;
#pragma omp parallel for
    for (long long c = 0; c < n; c++) {
        double out[Q19];
        orc19_collide_cell(f + c * Q19, tau, collision, out);
        memcpy(f + c * Q19, out, sizeof(out));
    }
}

/* Pull-streaming alone, f_i(x) <- f_i(x - xi_i), periodic, f in place. */
void orc19_stream(int32_t nx, int32_t ny, int32_t nz, double *f)
{
    orc19_init();
    const size_t n = (size_t)nx * ny * nz;
    double *C = (double *)malloc(n * Q19 * sizeof(double));
    memcpy(C, f, n * Q19 * sizeof(double));
    for (size_t c = 0; c < n; c++) {
        const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((size_t)nx * ny));
        for (int i = 0; i < Q19; i++) {
            const int xs = wrap19(x - xi19[i][0], nx), ys = wrap19(y - xi19[i][1], ny), zs = wrap19(z - xi19[i][2], nz);
            f[c * Q19 + i] = C[(((size_t)zs * ny + ys) * nx + xs) * Q19 + i];
        }
    }
    free(C);
}

/* nsteps of collide + pull-stream on an nx x ny x nz periodic box;
 * f is [nz][ny][nx][19], updated in place. */
void orc19_run(int32_t nx, int32_t ny, int32_t nz, double tau, int32_t collision, double *f, int32_t nsteps)
{
    orc19_init();
    const size_t n = (size_t)nx * ny * nz;
    double *C = (double *)malloc(n * Q19 * sizeof(double));
    for (int s = 0; s < nsteps; s++) {
#pragma omp parallel for
        for (long long c = 0; c < (long long)n; c++) orc19_collide_cell(f + c * Q19, tau, collision, C + c * Q19);
#pragma omp parallel for
        for (long long c = 0; c < (long long)n; c++) {
            const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((long long)nx * ny));
            for (int i = 0; i < Q19; i++) {
                const int xs = wrap19(x - xi19[i][0], nx), ys = wrap19(y - xi19[i][1], ny),
                          zs = wrap19(z - xi19[i][2], nz);
                f[c * Q19 + i] = C[(((size_t)zs * ny + ys) * nx + xs) * Q19 + i];
            }
        }
    }
    free(C);
}
