/*
 * vegas_oracle.h -- plain FP64 CPU reference ("oracle") for one Vegas iteration.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link or
 * call this code: it exists so that tests/, the smoke check and the benchmark's
 * CPU-baseline leg can check the HIP library against an independent, slow,
 * obviously correct implementation.  It shares no source with the HIP library.
 *
 * What it computes follows the paper's statement of the method (importance
 * sampling "as implemented in Vegas", sec. 2.2: a per-event stage followed by a
 * refinement of how the random numbers are generated once an integration pass
 * is finished), its toy integrands (sec. 3.1, Eqs. lepage, genzdisc and
 * productpeak) and its "value +- error" results (Table 1).  The paper prints
 * none of Vegas' formulas; those below are the published Vegas method it cites
 * (G.P. Lepage, J. Comput. Phys. 27 (1978) 192; Cornell CLNS-80/447 (1980)),
 * with every point where a choice had to be made listed in the design notes.
 * Random points come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC'11).
 *
 * Everything is FP64; sums are Neumaier-compensated and run in event order.
 */
#ifndef VEGAS_ORACLE_H
#define VEGAS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Integrand kinds (sec. 3.1). */
enum { VO_GAUSS = 0, VO_BIMODAL = 1, VO_GENZ_DISC = 2, VO_GENZ_PEAK = 3 };

/* One integration problem.  params layout per kind:
 *   VO_GAUSS     : a, mu[0..d-1]                      (1 + d values)
 *   VO_BIMODAL   : a, muA[0..d-1], muB[0..d-1]        (1 + 2d values)
 *   VO_GENZ_DISC : c[0..d-1], a[0..d-1]               (2d values)
 *   VO_GENZ_PEAK : c[0..d-1], a[0..d-1]               (2d values)            */
typedef struct {
    int32_t dim;
    int32_t n_bins;
    int32_t kind;
    int32_t problem;        /* p: goes into the Philox counter */
    uint64_t seed;          /* Philox key */
    double alpha;           /* damping exponent of the refinement */
    const double* params;
} vo_problem;

/* Philox4x32-10 bijection (SC'11, sec. 3). */
void vo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The d uniforms y in (0,1) of event e in iteration t of problem p. */
void vo_point(uint64_t seed, uint32_t t, uint32_t p, uint64_t e, int d, double* y);

/* Bin index b = floor(y N) and fractional position delta = y N - b. */
void vo_bin(double y, int n_bins, int32_t* b, double* delta);

/* Piecewise-linear map of y through the grid; returns the Jacobian weight. */
double vo_map(const double* edges, int d, int n_bins, const double* y,
              int32_t* b, double* delta, double* x);

/* Integrand value and its normalisation constant. */
double vo_norm(const vo_problem* pr);
double vo_integrand(const vo_problem* pr, const double* x);

/* d f / d theta for the Gaussian, theta = (mu[0..d-1], a). */
void vo_gauss_grad(const vo_problem* pr, const double* x, double* grad);

/* Accumulate S1 = sum f w, S2 = sum (f w)^2 and H[i][b] = sum (f w)^2 over
 * events with b_i = b, for events [e0, e0+n) of iteration t.  sums[0..1] and
 * H[d*N] are overwritten. */
void vo_accumulate(const vo_problem* pr, const double* edges, uint32_t t,
                   uint64_t e0, uint64_t n, double* sums, double* H);

/* The same accumulation over caller-supplied points y[n][d]. */
void vo_accumulate_points(const vo_problem* pr, const double* edges,
                          const double* y, uint64_t n, double* sums, double* H);

/* Per-event record (b, delta, x, w, f) for events [e0, e0+n):
 * out[n][3d+2] = b[0..d-1], delta[0..d-1], x[0..d-1], w, f. */
void vo_events(const vo_problem* pr, const double* edges, uint32_t t,
               uint64_t e0, uint64_t n, double* out);

/* Iteration estimate and its variance from S1, S2 over M events. */
void vo_iteration_stats(double S1, double S2, double M, double* I, double* var);

/* Grid refinement from the bin histograms H[d][N]. */
void vo_refine(const double* H, const double* edges_in, int d, int n_bins,
               double alpha, double* edges_out);

/* Damping function r(s) of the refinement, exposed for tests. */
double vo_damp(double s, double alpha);

/* Inverse-variance combination of m iteration results:
 * out[0] = I, out[1] = sigma, out[2] = chi^2/dof (NaN when m = 1). */
void vo_combine(const double* I, const double* var, int m, double* out);

/* Adjoint sums at fixed samples: G[j] = sum_e w_e d f/d theta_j (d+1 values)
 * and Gabs[j] = sum_e |w_e d f/d theta_j|, for a Gaussian problem. */
void vo_adjoint(const vo_problem* pr, const double* edges, uint32_t t,
                uint64_t e0, uint64_t n, double* G, double* Gabs);

/* A whole run: n_iter iterations of n_events each, starting at iteration
 * index t0 from edges (updated in place).  refine_after[k] != 0 refines
 * after iteration k; combine[k] != 0 includes it in the final combination.
 * iter_out[n_iter][2] = (I_t, var_t); final_out[3] = (I, sigma, chi2/dof);
 * H_last[d*N] = histograms of the last iteration. */
void vo_run(const vo_problem* pr, double* edges, uint32_t t0, int n_iter,
            uint64_t n_events, const int32_t* refine_after, const int32_t* combine,
            double* iter_out, double* final_out, double* H_last);

#ifdef __cplusplus
}
#endif

#endif
