/*
 * Oracle: brute-force history part of the split potentials (test infrastructure
 * only -- never linked into or called by the library).
 *
 * The paper splits the Laplace Green's function G(x) = -log|x|/(2 pi) in time
 * (Sec. 2, kernel splitting) as G = G_H[delta] + G_L[delta] with
 * G_L[delta](x) = E1(|x|^2/(4 delta))/(4 pi).  With Ein(z) = E1(z) + gamma + ln z
 * (entire), the history kernel is the smooth function
 *
 *     G_H[delta](d) = (gamma - ln(4 delta) - Ein(|d|^2/(4 delta))) / (4 pi).
 *
 * Near and far history together (Secs. 2-3, NH + FH = the whole history part)
 * are exactly the convolution of the quadrature sources with G_H[delta_1],
 * and the double layer uses its normal derivative in the source variable
 *
 *     K_D(x, y) = nu(y).(x - y) (1 - exp(-|x-y|^2/(4 delta))) / (2 pi |x-y|^2).
 *
 * This file evaluates those O(N_t * N_s) sums directly in double precision with
 * Neumaier-compensated accumulation, parallel over targets.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

static const double EULER_GAMMA = 0.57721566490153286061;
static const double PI = 3.14159265358979323846;

/* Exponential integral E1(z), z > 0, by its continued fraction (modified Lentz),
 * valid and fast for z >= 1: E1(z) = e^-z / (z + 1 - 1/(z + 3 - 4/(z + 5 - ...))). */
static double e1_cf(double z)
{
    const double tiny = 1e-300;
    double b = z + 1.0;
    double c = 1.0 / tiny;
    double d = 1.0 / b;
    double h = d;
    for (int i = 1; i < 1000; ++i) {
        double an = -(double)i * (double)i;
        b += 2.0;
        d = 1.0 / (an * d + b);
        c = b + an / c;
        double del = c * d;
        h *= del;
        if (fabs(del - 1.0) < 1e-17) break;
    }
    return h * exp(-z);
}

/* Ein(z) = sum_{n>=1} (-1)^{n+1} z^n / (n n!)  (entire; = E1 + gamma + ln z). */
double oracle_ein(double z)
{
    if (z < 2.0) {
        double term = z, sum = z;
        for (int n = 2; n < 60; ++n) {
            term *= -z / (double)n;           /* (-1)^{n+1} z^n / n! */
            double t = term / (double)n;
            sum += t;
            if (fabs(t) < 1e-18 * fabs(sum)) break;
        }
        return sum;
    }
    double e1 = (z > 745.0) ? 0.0 : e1_cf(z);
    return e1 + EULER_GAMMA + log(z);
}

/* G_H[delta](d) from |d|^2. */
double oracle_gh(double d2, double delta)
{
    double z = d2 / (4.0 * delta);
    if (z < 2.0)
        return (EULER_GAMMA - log(4.0 * delta) - oracle_ein(z)) / (4.0 * PI);
    /* gamma - ln 4delta - (E1 + gamma + ln z) = -ln d^2 - E1 */
    double e1 = (z > 745.0) ? 0.0 : e1_cf(z);
    return -(log(d2) + e1) / (4.0 * PI);
}

/* (1 - exp(-z)) / d^2 with its d -> 0 limit 1/(4 delta). */
static double kd_radial(double d2, double delta)
{
    if (d2 == 0.0) return 1.0 / (4.0 * delta);
    double z = d2 / (4.0 * delta);
    return -expm1(-z) / d2;
}

double oracle_kd(double dx, double dy, double nx, double ny, double delta)
{
    double d2 = dx * dx + dy * dy;
    return (nx * dx + ny * dy) * kd_radial(d2, delta) / (2.0 * PI);
}

typedef struct { double s, c; } acc_t;
static inline void acc_add(acc_t* a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

/*
 * History part at n_tgt targets.
 *   volume sources (n_src): c = f * w          -> outV (sum c G_H)
 *   boundary nodes (n_bnd): s = sigma * w_G     -> outS (sum s G_H)
 *                           m = mu * w_G, normal -> outD (sum m K_D)
 * Any of c, s, m may be NULL (its output is left untouched).
 */
void oracle_history(int64_t n_tgt, const double* tx, const double* ty,
                    int64_t n_src, const double* sx, const double* sy, const double* c,
                    int64_t n_bnd, const double* bx, const double* by,
                    const double* bnx, const double* bny,
                    const double* s, const double* m,
                    double delta, double* outV, double* outS, double* outD)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n_tgt; ++i) {
        const double x = tx[i], y = ty[i];
        if (c) {
            acc_t a = {0.0, 0.0};
            for (int64_t j = 0; j < n_src; ++j) {
                double dx = x - sx[j], dy = y - sy[j];
                acc_add(&a, c[j] * oracle_gh(dx * dx + dy * dy, delta));
            }
            outV[i] = a.s + a.c;
        }
        if (s) {
            acc_t a = {0.0, 0.0};
            for (int64_t j = 0; j < n_bnd; ++j) {
                double dx = x - bx[j], dy = y - by[j];
                acc_add(&a, s[j] * oracle_gh(dx * dx + dy * dy, delta));
            }
            outS[i] = a.s + a.c;
        }
        if (m) {
            acc_t a = {0.0, 0.0};
            for (int64_t j = 0; j < n_bnd; ++j) {
                double dx = x - bx[j], dy = y - by[j];
                acc_add(&a, m[j] * oracle_kd(dx, dy, bnx[j], bny[j], delta));
            }
            outD[i] = a.s + a.c;
        }
    }
}

/* Vectorised kernel values for tests: out[i] = G_H(d2[i]) or K_D. */
void oracle_gh_vec(int64_t n, const double* d2, double delta, double* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_gh(d2[i], delta);
}

void oracle_ein_vec(int64_t n, const double* z, double* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_ein(z[i]);
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
