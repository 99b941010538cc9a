/*
 * vegas_oracle.c -- plain FP64 CPU reference for one Vegas iteration.
 *
 * TEST INFRASTRUCTURE ONLY (see vegas_oracle.h).  Built with gcc,
 * -ffp-contract=off, no fast-math, single-threaded, so that every operation is
 * the IEEE double operation written here, in the order written here.
 */
#include "vegas_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11, sec. 3.2 and Table 2).
 * One round maps (c0, c1, c2, c3) with key (k0, k1) to
 *   (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0)),
 * and the key is bumped by the Weyl constants between rounds.            */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

void vo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Random points.  Event e of iteration t of problem p draws, for each group
 * j of four dimensions, Philox4x32-10 with
 *   counter = (e mod 2^32, e div 2^32, t, p*256 + j),  key = (seed mod 2^32, seed div 2^32),
 * and dimension i uses word i mod 4 of group j = i div 4.  A word k becomes
 * the uniform y = (k + 1/2) / 2^32, which lies strictly inside (0,1).      */
void vo_point(uint64_t seed, uint32_t t, uint32_t p, uint64_t e, int d, double* y)
{
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    for (int j = 0; 4 * j < d; ++j) {
        uint32_t ctr[4] = { (uint32_t)(e & 0xffffffffu), (uint32_t)(e >> 32), t,
                            p * 256u + (uint32_t)j };
        uint32_t k[4];
        vo_philox4x32_10(ctr, key, k);
        for (int q = 0; q < 4 && 4 * j + q < d; ++q)
            y[4 * j + q] = ((double)k[q] + 0.5) / 4294967296.0;
    }
}

/* Bin b = floor(y N), delta = y N - b.  For y = (k + 1/2)/2^32 and N < 256
 * the product y N has at most 41 significant bits, so it, the floor and the
 * difference are exact in FP64. */
void vo_bin(double y, int n_bins, int32_t* b, double* delta)
{
    double yn = y * (double)n_bins;
    double fb = floor(yn);
    *b = (int32_t)fb;
    *delta = yn - fb;
}

/* ------------------------------------------------------------------------ */
/* Vegas map (Lepage 1978, sec. 2): each dimension has N bins with edges
 * 0 = E_0 < E_1 < ... < E_N = 1; the uniform y falls into bin b at relative
 * position delta, is sent to x = E_b + delta (E_{b+1} - E_b), and the change
 * of variables has Jacobian N (E_{b+1} - E_b) in that dimension.          */
double vo_map(const double* edges, int d, int n_bins, const double* y,
              int32_t* b, double* delta, double* x)
{
    double w = 1.0;
    for (int i = 0; i < d; ++i) {
        const double* E = edges + (size_t)i * (n_bins + 1);
        vo_bin(y[i], n_bins, &b[i], &delta[i]);
        double lo = E[b[i]];
        double width = E[b[i] + 1] - E[b[i]];
        x[i] = lo + delta[i] * width;
        w = w * ((double)n_bins * width);
    }
    return w;
}

/* ------------------------------------------------------------------------ */
/* Integrands of sec. 3.1.
 * Gaussian (Eq. lepage): f = nu exp(-sum (x_i - mu_i)^2 / a^2), nu = (a sqrt(pi))^-d.
 * Bimodal: f = nu/2 [exp(-sum (x_i - muA_i)^2/a^2) + exp(-sum (x_i - muB_i)^2/a^2)].
 * Genz discontinuous (Eq. genzdisc): 0 if any x_i <= a_i, else nu exp(sum c_i x_i),
 *   nu = prod c_i / (e^{c_i} - e^{c_i a_i}).
 * Genz product peak (Eq. productpeak): nu prod 1/(c_i^-2 + (x_i - a_i)^2),
 *   nu = 1 / prod c_i [atan(c_i (1 - a_i)) + atan(c_i a_i)].
 * nu makes each integral over [0,1]^d equal to one, except the two Gaussian
 * forms, whose nu is the whole-space normalisation (integral erf products). */
double vo_norm(const vo_problem* pr)
{
    const int d = pr->dim;
    const double* q = pr->params;
    const double pi = 3.14159265358979323846;
    switch (pr->kind) {
    case VO_GAUSS:
    case VO_BIMODAL:
        return pow(q[0] * sqrt(pi), (double)(-d));
    case VO_GENZ_DISC: {
        double nu = 1.0;
        for (int i = 0; i < d; ++i) {
            double c = q[i], a = q[d + i];
            nu = nu * (c / (exp(c) - exp(c * a)));
        }
        return nu;
    }
    case VO_GENZ_PEAK: {
        double z = 1.0;
        for (int i = 0; i < d; ++i) {
            double c = q[i], a = q[d + i];
            z = z * (c * (atan(c * (1.0 - a)) + atan(c * a)));
        }
        return 1.0 / z;
    }
    }
    return NAN;
}

static double integrand_nu(const vo_problem* pr, double nu, const double* x)
{
    const int d = pr->dim;
    const double* q = pr->params;
    switch (pr->kind) {
    case VO_GAUSS: {
        double a = q[0], s = 0.0;
        for (int i = 0; i < d; ++i) {
            double u = x[i] - q[1 + i];
            s = s + u * u;
        }
        return nu * exp(-s / (a * a));
    }
    case VO_BIMODAL: {
        double a = q[0], sa = 0.0, sb = 0.0;
        for (int i = 0; i < d; ++i) {
            double u = x[i] - q[1 + i];
            double v = x[i] - q[1 + d + i];
            sa = sa + u * u;
            sb = sb + v * v;
        }
        return 0.5 * nu * (exp(-sa / (a * a)) + exp(-sb / (a * a)));
    }
    case VO_GENZ_DISC: {
        double s = 0.0;
        for (int i = 0; i < d; ++i) {
            if (x[i] <= q[d + i]) return 0.0;
            s = s + q[i] * x[i];
        }
        return nu * exp(s);
    }
    case VO_GENZ_PEAK: {
        double prod = 1.0;
        for (int i = 0; i < d; ++i) {
            double c = q[i], u = x[i] - q[d + i];
            prod = prod * (1.0 / (1.0 / (c * c) + u * u));
        }
        return nu * prod;
    }
    }
    return NAN;
}

double vo_integrand(const vo_problem* pr, const double* x)
{
    return integrand_nu(pr, vo_norm(pr), x);
}

/* Gaussian derivatives: df/dmu_j = f 2 (x_j - mu_j)/a^2 and, since nu is
 * proportional to a^-d, df/da = f (2 sum (x_i - mu_i)^2 / a^3 - d / a). */
void vo_gauss_grad(const vo_problem* pr, const double* x, double* grad)
{
    const int d = pr->dim;
    const double a = pr->params[0];
    const double f = vo_integrand(pr, x);
    double s = 0.0;
    for (int j = 0; j < d; ++j) {
        double u = x[j] - pr->params[1 + j];
        s = s + u * u;
        grad[j] = f * 2.0 * u / (a * a);
    }
    grad[d] = f * (2.0 * s / (a * a * a) - (double)d / a);
}

/* ------------------------------------------------------------------------ */
/* Neumaier's compensated summation. */
typedef struct { double s, c; } vo_sum;

static void vo_sum_add(vo_sum* a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double vo_sum_value(const vo_sum* a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* Per-iteration accumulators (Lepage 1978 sec. 3; 1980): the estimate is the
 * mean of v = f(x) w over the M events, its variance follows from the sum of
 * v^2, and the grid is driven by the per-dimension, per-bin sums of v^2.   */
static void accumulate_from(const vo_problem* pr, const double* edges,
                            uint32_t t, uint64_t e0, const double* ypts,
                            uint64_t n, double* sums, double* H)
{
    const int d = pr->dim, N = pr->n_bins;
    double* y = malloc(sizeof(double) * d);
    double* x = malloc(sizeof(double) * d);
    double* delta = malloc(sizeof(double) * d);
    int32_t* b = malloc(sizeof(int32_t) * d);
    vo_sum* h = calloc((size_t)d * N, sizeof(vo_sum));
    vo_sum s1 = {0, 0}, s2 = {0, 0};
    const double nu = vo_norm(pr);

    for (uint64_t k = 0; k < n; ++k) {
        if (ypts)
            memcpy(y, ypts + k * d, sizeof(double) * d);
        else
            vo_point(pr->seed, t, (uint32_t)pr->problem, e0 + k, d, y);
        double w = vo_map(edges, d, N, y, b, delta, x);
        double f = integrand_nu(pr, nu, x);
        double v = f * w;
        double v2 = v * v;
        vo_sum_add(&s1, v);
        vo_sum_add(&s2, v2);
        for (int i = 0; i < d; ++i)
            vo_sum_add(&h[(size_t)i * N + b[i]], v2);
    }
    sums[0] = vo_sum_value(&s1);
    sums[1] = vo_sum_value(&s2);
    for (size_t k = 0; k < (size_t)d * N; ++k)
        H[k] = vo_sum_value(&h[k]);
    free(y); free(x); free(delta); free(b); free(h);
}

void vo_accumulate(const vo_problem* pr, const double* edges, uint32_t t,
                   uint64_t e0, uint64_t n, double* sums, double* H)
{
    accumulate_from(pr, edges, t, e0, NULL, n, sums, H);
}

void vo_accumulate_points(const vo_problem* pr, const double* edges,
                          const double* y, uint64_t n, double* sums, double* H)
{
    accumulate_from(pr, edges, 0, 0, y, n, sums, H);
}

void vo_events(const vo_problem* pr, const double* edges, uint32_t t,
               uint64_t e0, uint64_t n, double* out)
{
    const int d = pr->dim, N = pr->n_bins;
    double* y = malloc(sizeof(double) * d);
    double* x = malloc(sizeof(double) * d);
    double* delta = malloc(sizeof(double) * d);
    int32_t* b = malloc(sizeof(int32_t) * d);
    for (uint64_t k = 0; k < n; ++k) {
        double* row = out + k * (size_t)(3 * d + 2);
        vo_point(pr->seed, t, (uint32_t)pr->problem, e0 + k, d, y);
        double w = vo_map(edges, d, N, y, b, delta, x);
        double f = vo_integrand(pr, x);
        for (int i = 0; i < d; ++i) {
            row[i] = (double)b[i];
            row[d + i] = delta[i];
            row[2 * d + i] = x[i];
        }
        row[3 * d] = w;
        row[3 * d + 1] = f;
    }
    free(y); free(x); free(delta); free(b);
}

/* I_t = S1 / M;  var_t = (S2 / M - I_t^2) / (M - 1): the sample variance of
 * v divided by M, i.e. the variance of the mean (Lepage 1978, eq. for sigma^2). */
void vo_iteration_stats(double S1, double S2, double M, double* I, double* var)
{
    double mean = S1 / M;
    *I = mean;
    *var = (S2 / M - mean * mean) / (M - 1.0);
}

/* ------------------------------------------------------------------------ */
/* Refinement (Lepage 1978 sec. 3, in the continuous form of the 1980 program).
 * For each dimension, with d_b the histogram of bin b:
 *  1. if all d_b are zero the dimension is left as it is;
 *  2. smooth: s_b = mean of d over bins b-1, b, b+1 that exist;
 *  3. normalise: s_b / sum s;
 *  4. damp: r_b = ((s_b - 1) / ln s_b)^alpha, with r = 0 at s = 0 and r = 1 at s = 1;
 *  5. rebin: spread r_b uniformly over old bin b and place new edge k where
 *     the cumulative amount of r first reaches k/N of its total; the end
 *     edges 0 and 1 are kept.                                               */
double vo_damp(double s, double alpha)
{
    if (s == 0.0) return 0.0;
    if (s == 1.0) return 1.0;
    return pow((s - 1.0) / log(s), alpha);
}

void vo_refine(const double* H, const double* edges_in, int d, int n_bins,
               double alpha, double* edges_out)
{
    const int N = n_bins;
    double* s = malloc(sizeof(double) * N);
    double* r = malloc(sizeof(double) * N);
    for (int i = 0; i < d; ++i) {
        const double* h = H + (size_t)i * N;
        const double* E = edges_in + (size_t)i * (N + 1);
        double* Eo = edges_out + (size_t)i * (N + 1);

        double total = 0.0;
        for (int b = 0; b < N; ++b) total = total + h[b];

        s[0] = (h[0] + h[1]) / 2.0;
        for (int b = 1; b < N - 1; ++b) s[b] = (h[b - 1] + h[b] + h[b + 1]) / 3.0;
        s[N - 1] = (h[N - 2] + h[N - 1]) / 2.0;

        double ssum = 0.0;
        for (int b = 0; b < N; ++b) ssum = ssum + s[b];

        /* nothing to adapt to: an empty histogram, or one whose total is not
         * a finite number (the dimension keeps its grid) */
        if (!(total > 0.0 && total <= DBL_MAX && ssum > 0.0 && ssum <= DBL_MAX)) {
            for (int k = 0; k <= N; ++k) Eo[k] = E[k];
            continue;
        }

        double rsum = 0.0;
        for (int b = 0; b < N; ++b) {
            r[b] = vo_damp(s[b] / ssum, alpha);
            rsum = rsum + r[b];
        }

        Eo[0] = E[0];
        Eo[N] = E[N];
        int b = 0;
        double acc = 0.0;            /* amount of r in bins 0..b-1 */
        for (int k = 1; k < N; ++k) {
            double level = (double)k * rsum / (double)N;
            while (b < N - 1 && acc + r[b] < level) {
                acc = acc + r[b];
                b = b + 1;
            }
            Eo[k] = E[b] + (level - acc) / r[b] * (E[b + 1] - E[b]);
        }
    }
    free(s); free(r);
}

/* ------------------------------------------------------------------------ */
/* Combination of iterations into "value +- error" (Table 1): the
 * inverse-variance weighted mean, its error, and chi^2 per degree of freedom
 * of the iterations around it (Lepage 1978 sec. 3).                       */
void vo_combine(const double* I, const double* var, int m, double* out)
{
    double sw = 0.0, swi = 0.0;
    for (int k = 0; k < m; ++k) {
        sw = sw + 1.0 / var[k];
        swi = swi + I[k] / var[k];
    }
    double mean = swi / sw;
    double chi2 = 0.0;
    for (int k = 0; k < m; ++k)
        chi2 = chi2 + (I[k] - mean) * (I[k] - mean) / var[k];
    out[0] = mean;
    out[1] = sqrt(1.0 / sw);
    out[2] = (m > 1) ? chi2 / (double)(m - 1) : NAN;
}

/* ------------------------------------------------------------------------ */
/* Adjoint at fixed samples and a fixed grid: with the points and the grid
 * held fixed, d/d theta of the estimate (1/M) sum f(x_e; theta) w_e is
 * (1/M) sum w_e df/d theta (x_e).  Returned unscaled (no 1/M).              */
void vo_adjoint(const vo_problem* pr, const double* edges, uint32_t t,
                uint64_t e0, uint64_t n, double* G, double* Gabs)
{
    const int d = pr->dim, N = pr->n_bins;
    double* y = malloc(sizeof(double) * d);
    double* x = malloc(sizeof(double) * d);
    double* delta = malloc(sizeof(double) * d);
    double* g = malloc(sizeof(double) * (d + 1));
    int32_t* b = malloc(sizeof(int32_t) * d);
    vo_sum* acc = calloc((size_t)d + 1, sizeof(vo_sum));
    vo_sum* aabs = calloc((size_t)d + 1, sizeof(vo_sum));
    for (uint64_t k = 0; k < n; ++k) {
        vo_point(pr->seed, t, (uint32_t)pr->problem, e0 + k, d, y);
        double w = vo_map(edges, d, N, y, b, delta, x);
        vo_gauss_grad(pr, x, g);
        for (int j = 0; j <= d; ++j) {
            vo_sum_add(&acc[j], w * g[j]);
            vo_sum_add(&aabs[j], fabs(w * g[j]));
        }
    }
    for (int j = 0; j <= d; ++j) {
        G[j] = vo_sum_value(&acc[j]);
        Gabs[j] = vo_sum_value(&aabs[j]);
    }
    free(y); free(x); free(delta); free(g); free(b); free(acc); free(aabs);
}

/* ------------------------------------------------------------------------ */
/* A whole run: iterate, optionally refine after each iteration, combine the
 * flagged iterations. */
void vo_run(const vo_problem* pr, double* edges, uint32_t t0, int n_iter,
            uint64_t n_events, const int32_t* refine_after, const int32_t* combine,
            double* iter_out, double* final_out, double* H_last)
{
    const int d = pr->dim, N = pr->n_bins;
    double* H = malloc(sizeof(double) * (size_t)d * N);
    double* En = malloc(sizeof(double) * (size_t)d * (N + 1));
    double* Ic = malloc(sizeof(double) * (n_iter > 0 ? n_iter : 1));
    double* Vc = malloc(sizeof(double) * (n_iter > 0 ? n_iter : 1));
    int m = 0;
    for (int k = 0; k < n_iter; ++k) {
        double sums[2];
        vo_accumulate(pr, edges, t0 + (uint32_t)k, 0, n_events, sums, H);
        vo_iteration_stats(sums[0], sums[1], (double)n_events,
                           &iter_out[2 * k], &iter_out[2 * k + 1]);
        if (combine[k]) {
            Ic[m] = iter_out[2 * k];
            Vc[m] = iter_out[2 * k + 1];
            m = m + 1;
        }
        if (refine_after[k]) {
            vo_refine(H, edges, d, N, pr->alpha, En);
            memcpy(edges, En, sizeof(double) * (size_t)d * (N + 1));
        }
    }
    if (m > 0)
        vo_combine(Ic, Vc, m, final_out);
    else
        final_out[0] = final_out[1] = final_out[2] = NAN;
    if (H_last) memcpy(H_last, H, sizeof(double) * (size_t)d * N);
    free(H); free(En); free(Ic); free(Vc);
}
