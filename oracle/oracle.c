/*
 * oracle.c -- plain, serial FP64 CPU reference for the long-range MD hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker of the GPU library: only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 * It shares no code, header, table or constant with the HIP path.
 *
 * What it computes (Rocha Filho, "Molecular dynamics for long-range interacting
 * systems on Graphic Processing Units"; equations numbered as in the paper):
 *
 *   models       Ring (Sec. 2, eq. 1), HMF (Sec. 2, eq. 2), 2D self-gravitating
 *                (Sec. 2, eq. 3); unit masses, 1/N coupling.
 *   forces       f_i = -dV/dq_i written out as the plain all-pairs sum, i outer,
 *                j ascending inner, plain FP64 '+=' (Sec. 3.2: eqs. 8 and 9 give
 *                the Ring pair force; the 2D pair force is the gradient of eq. 3).
 *                HMF uses the O(N) magnetization form (Sec. 3.1, eqs. 6 and 7); the
 *                O(N^2) pair sum is kept as a pin.
 *   integrator   the 4th-order Yoshida composition of Sec. 3, eq. 4, as a
 *                kick-drift sequence with the last force of a step reused as the
 *                first of the next.
 *   energies     K = 1/2 sum p^2; V exactly per the Hamiltonians over i<j; HMF also
 *                through eq. 5.  Large sums are Neumaier-compensated.
 *   adjoint      Hessian-vector products of V and the reverse-mode derivative of
 *                the integrator (recompute the forward steps, undo kicks and drifts
 *                in reverse order); not part of the paper, which integrates forward
 *                only -- derivatives of the same discrete map.
 *
 * Readings of the paper taken here (each is pinned by the tests):
 *   - Ring force sign: eqs. 8 and 9 print +dV/dtheta_i; the force used is
 *     -dV/dtheta_i, i.e. f_ij = -(1/(2 sqrt2 N)) sin(ti-tj) / (1-cos(ti-tj)+eps)^{3/2}.
 *   - The 2D pair force is -(2/N) (r_i - r_j) / (|r_i - r_j|^2 + eps); log is natural.
 *   - Yoshida constants (not printed in the paper): the triple-jump composition of
 *     the kick-drift-kick leapfrog, w1 = 1/(2 - 2^{1/3}), w0 = -2^{1/3}/(2 - 2^{1/3});
 *     B0 = w1/2, B1 = (w0 + w1)/2, D0 = w1, D1 = w0.
 *   - The final kick of a step uses the force at the new positions, and that force
 *     is carried into the next step (the step list of Sec. 3 names f^(I) for that
 *     kick and f^(II) for the carried force; only the reading taken here is
 *     time-reversible, 4th order, and needs three force evaluations per step).
 *   - The self pair j = i contributes nothing and is skipped.
 *
 * Layout: q, p, f are FP64 structure-of-arrays [d][n] (d = 2 for 2D gravity: x row
 * then y row; d = 1 otherwise), host memory owned by the caller.
 *
 * Threads: an optional OpenMP loop over the outer particle index i.  Each i's inner
 * sum stays serial and every reduction over i is done serially afterwards, so the
 * results are bitwise identical for any thread count.
 *
 * Build: gcc -O2 -fPIC -shared -fopenmp -ffp-contract=off (no fast-math).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_HMF 0
#define OR_RING 1
#define OR_GRAV2D 2

static int or_dims(int model) { return model == OR_GRAV2D ? 2 : 1; }

static int or_model_ok(int model) { return model == OR_HMF || model == OR_RING || model == OR_GRAV2D; }

/* ---------------------------------------------------------------- threads -- */

void or_set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int or_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------- compensated sums -- */

/* Neumaier's variant of Kahan summation: s + c carries the running sum. */
typedef struct { double s, c; } or_acc;

static void acc_add(or_acc *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else                       a->c += (x - t) + a->s;
    a->s = t;
}

static double acc_val(const or_acc *a) { return a->s + a->c; }

static double or_sum(const double *x, long n)
{
    or_acc a = {0.0, 0.0};
    for (long i = 0; i < n; ++i) acc_add(&a, x[i]);
    return acc_val(&a);
}

/* ------------------------------------------------------- Yoshida constants -- */

/* c = {B0, B1, D0, D1} of eq. 4 (triple jump of the leapfrog). */
void or_yoshida(double c[4])
{
    double cb = cbrt(2.0);
    double w1 = 1.0 / (2.0 - cb);
    double w0 = -cb / (2.0 - cb);
    c[0] = 0.5 * w1;
    c[1] = 0.5 * (w0 + w1);
    c[2] = w1;
    c[3] = w0;
}

/* ------------------------------------------------------------ pair forces -- */

/* Ring: -dV/dtheta_i of eq. 1, the difference form of eq. 8 (sign corrected). */
static double ring_row(long n, double eps, const double *th, long i)
{
    double s = 0.0;
    for (long j = 0; j < n; ++j) {
        if (j == i) continue;
        double d = th[i] - th[j];
        double u = 1.0 - cos(d) + eps;
        s += sin(d) / (u * sqrt(u));
    }
    return -s / (2.0 * sqrt(2.0) * (double)n);
}

/* 2D gravity: -dV/dr_i of eq. 3. */
static void grav2d_row(long n, double eps, const double *x, const double *y, long i,
                       double *fx, double *fy)
{
    double sx = 0.0, sy = 0.0;
    for (long j = 0; j < n; ++j) {
        if (j == i) continue;
        double dx = x[i] - x[j];
        double dy = y[i] - y[j];
        double w = 1.0 / (dx * dx + dy * dy + eps);
        sx += dx * w;
        sy += dy * w;
    }
    *fx = -2.0 * sx / (double)n;
    *fy = -2.0 * sy / (double)n;
}

/* HMF as the plain pair sum -dV/dtheta_i of eq. 2 (kept as the pin of the O(N) form). */
static double hmf_pair_row(long n, const double *th, long i)
{
    double s = 0.0;
    for (long j = 0; j < n; ++j) {
        if (j == i) continue;
        s += sin(th[i] - th[j]);
    }
    return -s / (double)n;
}

/* Magnetization of eq. 7: m[0] = Mx, m[1] = My. */
void or_magnetization(long n, const double *th, double m[2])
{
    or_acc ax = {0.0, 0.0}, ay = {0.0, 0.0};
    for (long i = 0; i < n; ++i) {
        acc_add(&ax, cos(th[i]));
        acc_add(&ay, sin(th[i]));
    }
    m[0] = acc_val(&ax) / (double)n;
    m[1] = acc_val(&ay) / (double)n;
}

/* HMF force through eqs. 6 and 7: f_i = cos(ti) My - sin(ti) Mx. */
static void hmf_force(long n, const double *th, double *f)
{
    double m[2];
    or_magnetization(n, th, m);
    long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) f[i] = cos(th[i]) * m[1] - sin(th[i]) * m[0];
}

/* f = force(q) for all particles.  Returns 0, or -1 on bad arguments. */
int or_force(int model, long n, double eps, const double *q, double *f)
{
    if (!or_model_ok(model) || n < 0) return -1;
    if (n == 0) return 0;
    long i;
    if (model == OR_HMF) {
        hmf_force(n, q, f);
    } else if (model == OR_RING) {
#pragma omp parallel for schedule(dynamic, 16)
        for (i = 0; i < n; ++i) f[i] = ring_row(n, eps, q, i);
    } else {
#pragma omp parallel for schedule(dynamic, 16)
        for (i = 0; i < n; ++i) grav2d_row(n, eps, q, q + n, i, &f[i], &f[n + i]);
    }
    return 0;
}

/* Force on a subset of particles: f_rows is [d][nrows], row k is particle rows[k]. */
int or_force_rows(int model, long n, double eps, const double *q,
                  const long *rows, long nrows, double *f_rows)
{
    if (!or_model_ok(model) || n < 0 || nrows < 0) return -1;
    for (long k = 0; k < nrows; ++k)
        if (rows[k] < 0 || rows[k] >= n) return -1;
    long k;
    if (model == OR_HMF) {
        double m[2];
        or_magnetization(n, q, m);
        for (k = 0; k < nrows; ++k) {
            double t = q[rows[k]];
            f_rows[k] = cos(t) * m[1] - sin(t) * m[0];
        }
    } else if (model == OR_RING) {
#pragma omp parallel for schedule(dynamic, 4)
        for (k = 0; k < nrows; ++k) f_rows[k] = ring_row(n, eps, q, rows[k]);
    } else {
#pragma omp parallel for schedule(dynamic, 4)
        for (k = 0; k < nrows; ++k)
            grav2d_row(n, eps, q, q + n, rows[k], &f_rows[k], &f_rows[nrows + k]);
    }
    return 0;
}

/* HMF force as the O(N^2) pair sum (pin of the mean-field identity). */
int or_hmf_force_pairs(long n, const double *th, double *f)
{
    if (n < 0) return -1;
    long i;
#pragma omp parallel for schedule(dynamic, 16)
    for (i = 0; i < n; ++i) f[i] = hmf_pair_row(n, th, i);
    return 0;
}

/* ------------------------------------------------------------- integrator -- */

static void kick(long len, double *p, const double *f, double h)
{
    for (long k = 0; k < len; ++k) p[k] += h * f[k];
}

static void drift(long len, double *q, const double *p, double h)
{
    for (long k = 0; k < len; ++k) q[k] += h * p[k];
}

/*
 * nsteps Yoshida steps of size dt (eq. 4), in place.  On entry f must hold
 * force(q); on exit it holds force(q_final).  Three force evaluations per step.
 */
int or_step(int model, long n, double eps, double *q, double *p, double *f,
            double dt, long nsteps)
{
    if (!or_model_ok(model) || n < 0 || nsteps < 0) return -1;
    double c[4];
    or_yoshida(c);
    const double B0 = c[0], B1 = c[1], D0 = c[2], D1 = c[3];
    long len = (long)or_dims(model) * n;
    for (long s = 0; s < nsteps; ++s) {
        kick(len, p, f, B0 * dt);
        drift(len, q, p, D0 * dt);
        or_force(model, n, eps, q, f);
        kick(len, p, f, B1 * dt);
        drift(len, q, p, D1 * dt);
        or_force(model, n, eps, q, f);
        kick(len, p, f, B1 * dt);
        drift(len, q, p, D0 * dt);
        or_force(model, n, eps, q, f);
        kick(len, p, f, B0 * dt);
    }
    return 0;
}

/* --------------------------------------------------------------- energies -- */

double or_kinetic(int model, long n, const double *p)
{
    if (!or_model_ok(model) || n <= 0) return 0.0;
    or_acc a = {0.0, 0.0};
    long len = (long)or_dims(model) * n;
    for (long k = 0; k < len; ++k) acc_add(&a, p[k] * p[k]);
    return 0.5 * acc_val(&a);
}

/* Potential energy exactly per the Hamiltonians (pairs i < j). */
double or_potential(int model, long n, double eps, const double *q)
{
    if (!or_model_ok(model) || n <= 0) return 0.0;
    if (model == OR_HMF) {
        double m[2];
        or_magnetization(n, q, m);
        return 0.5 * (double)n * (1.0 - m[0] * m[0] - m[1] * m[1]);
    }
    double *row = (double *)malloc(sizeof(double) * (size_t)n);
    if (!row) return NAN;
    long i;
#pragma omp parallel for schedule(dynamic, 16)
    for (i = 0; i < n; ++i) {
        or_acc a = {0.0, 0.0};
        if (model == OR_RING) {
            for (long j = i + 1; j < n; ++j)
                acc_add(&a, 1.0 / (sqrt(2.0) * sqrt(1.0 - cos(q[i] - q[j]) + eps)));
            row[i] = -acc_val(&a);
        } else {
            const double *x = q, *y = q + n;
            for (long j = i + 1; j < n; ++j) {
                double dx = x[i] - x[j], dy = y[i] - y[j];
                acc_add(&a, log(dx * dx + dy * dy + eps));
            }
            row[i] = acc_val(&a);
        }
    }
    double v = or_sum(row, n) / (double)n;
    free(row);
    return v;
}

/* HMF potential as the pair sum of eq. 2 (pin of eq. 5). */
double or_hmf_potential_pairs(long n, const double *th)
{
    if (n <= 0) return 0.0;
    double *row = (double *)malloc(sizeof(double) * (size_t)n);
    if (!row) return NAN;
    long i;
#pragma omp parallel for schedule(dynamic, 16)
    for (i = 0; i < n; ++i) {
        or_acc a = {0.0, 0.0};
        for (long j = i + 1; j < n; ++j) acc_add(&a, 1.0 - cos(th[i] - th[j]));
        row[i] = acc_val(&a);
    }
    double v = or_sum(row, n) / (double)n;
    free(row);
    return v;
}

/* out[0] = K, out[1] = V, out[2] = E = K + V.  Returns 0, or -1 on bad arguments. */
int or_energy(int model, long n, double eps, const double *q, const double *p, double out[3])
{
    if (!or_model_ok(model) || n < 0) return -1;
    out[0] = or_kinetic(model, n, p);
    out[1] = or_potential(model, n, eps, q);
    out[2] = out[0] + out[1];
    return 0;
}

/* ------------------------------------------------------------------ adjoint -- */
/*
 * Hessian-vector product out = H(q) w, H = second derivatives of the potential V
 * of eqs. 1-3 (the force is -grad V, so the Jacobian of the force is -H).  For a
 * pair potential V = sum_{i<j} phi(q_i - q_j) the product is
 *     (H w)_i = sum_{j != i} phi''(q_i - q_j) (w_i - w_j),
 * with phi'' the 1x1 (angles) or 2x2 (2D) second derivative of the pair term:
 *   Ring  phi(d) = -(1/(sqrt2 N)) u^{-1/2}, u = 1 - cos d + eps:
 *         phi''(d) = (1/(2 sqrt2 N)) [cos d u^{-3/2} - (3/2) sin^2 d u^{-5/2}]
 *   HMF   phi(d) = (1/N)(1 - cos d):  phi''(d) = (1/N) cos d
 *   2D    phi(r) = (1/N) log(|r|^2 + eps), s = |r|^2 + eps:
 *         phi''(r) = (2/N) [I/s - 2 r r^T / s^2]
 */
int or_hvp(int model, long n, double eps, const double *q, const double *w, double *out)
{
    if (!or_model_ok(model) || n < 0) return -1;
    long i;
    if (model == OR_GRAV2D) {
        const double *x = q, *y = q + n, *wx = w, *wy = w + n;
#pragma omp parallel for schedule(dynamic, 16)
        for (i = 0; i < n; ++i) {
            double ax = 0.0, ay = 0.0;
            for (long j = 0; j < n; ++j) {
                if (j == i) continue;
                double dx = x[i] - x[j], dy = y[i] - y[j];
                double s = dx * dx + dy * dy + eps;
                double ux = wx[i] - wx[j], uy = wy[i] - wy[j];
                double rdotu = dx * ux + dy * uy;
                ax += ux / s - 2.0 * dx * rdotu / (s * s);
                ay += uy / s - 2.0 * dy * rdotu / (s * s);
            }
            out[i] = 2.0 * ax / (double)n;
            out[n + i] = 2.0 * ay / (double)n;
        }
    } else {
#pragma omp parallel for schedule(dynamic, 16)
        for (i = 0; i < n; ++i) {
            double a = 0.0;
            for (long j = 0; j < n; ++j) {
                if (j == i) continue;
                double d = q[i] - q[j];
                double h;
                if (model == OR_RING) {
                    double u = 1.0 - cos(d) + eps;
                    h = (cos(d) / (u * sqrt(u)) - 1.5 * sin(d) * sin(d) / (u * u * sqrt(u))) /
                        (2.0 * sqrt(2.0) * (double)n);
                } else {
                    h = cos(d) / (double)n;
                }
                a += h * (w[i] - w[j]);
            }
            out[i] = a;
        }
    }
    return 0;
}

/*
 * Reverse-mode derivative (vector-Jacobian product) of nsteps Yoshida steps
 * (eq. 4) started from (q0, p0): on entry (lq, lp) are the adjoints dJ/dq, dJ/dp
 * of some J at the final state; on exit they are dJ/dq0, dJ/dp0.  The forward
 * steps are recomputed and every position at which a kick evaluates the force is
 * kept; the kicks and drifts are then undone in reverse order:
 *     drift q += a p:        lp += a lq
 *     kick  p += h F(q):     lq -= h H(q) lp        (F = -grad V)
 */
int or_step_vjp(int model, long n, double eps, const double *q0, const double *p0, double dt, long nsteps,
                double *lq, double *lp)
{
    if (!or_model_ok(model) || n < 0 || nsteps < 0) return -1;
    double c[4];
    or_yoshida(c);
    const double kick_w[4] = {c[0], c[1], c[1], c[0]};
    const double drift_w[3] = {c[2], c[3], c[2]};
    long len = (long)or_dims(model) * n;
    /* positions at the 4 kicks of every step: (nsteps * 4) x len */
    double *qs = (double *)malloc(sizeof(double) * (size_t)len * (size_t)(4 * nsteps + 1));
    double *q = (double *)malloc(sizeof(double) * (size_t)len);
    double *p = (double *)malloc(sizeof(double) * (size_t)len);
    double *f = (double *)malloc(sizeof(double) * (size_t)len);
    double *hw = (double *)malloc(sizeof(double) * (size_t)len);
    if (!qs || !q || !p || !f || !hw) {
        free(qs); free(q); free(p); free(f); free(hw);
        return -1;
    }
    memcpy(q, q0, sizeof(double) * (size_t)len);
    memcpy(p, p0, sizeof(double) * (size_t)len);
    for (long s = 0; s < nsteps; ++s) {
        for (int k = 0; k < 4; ++k) {
            memcpy(qs + (size_t)(4 * s + k) * len, q, sizeof(double) * (size_t)len);
            or_force(model, n, eps, q, f);
            kick(len, p, f, kick_w[k] * dt);
            if (k < 3) drift(len, q, p, drift_w[k] * dt);
        }
    }
    for (long s = nsteps - 1; s >= 0; --s) {
        for (int k = 3; k >= 0; --k) {
            if (k < 3) /* undo drift k: q += a p */
                for (long m = 0; m < len; ++m) lp[m] += drift_w[k] * dt * lq[m];
            or_hvp(model, n, eps, qs + (size_t)(4 * s + k) * len, lp, hw);
            for (long m = 0; m < len; ++m) lq[m] -= kick_w[k] * dt * hw[m];
        }
    }
    free(qs); free(q); free(p); free(f); free(hw);
    return 0;
}
