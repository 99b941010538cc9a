"""Example user integrands: HIP device source for ``Vegas(..., source=...)``
(compiled at run time for gfx950; see vegas_init_user in include/vegas.h).

Each source defines ``__device__ vegas_real vegas_integrand(const vegas_real*
x, int dim, const double* params)`` on [0,1)^dim; vegas_real is double in an
FP64 context and float in an FP32-mixed one.  These examples do their own
arithmetic in FP64 either way.

  GAUSSIAN        the Gaussian of sec. 3.1 written out by hand:
                  nu exp(-sum (x_i - mu_i)^2 / a^2), nu = (a sqrt(pi))^-d;
                  params = a, mu[0..d-1] (the built-in VEGAS_GAUSS layout)
  OSCILLATORY     Genz's oscillatory family: cos(2 pi u + sum c_i x_i);
                  params = u, c[0..d-1]; integral
                  Re[exp(2 pi i u) prod (exp(i c_j) - 1) / (i c_j)]
  SINE_PRODUCT    prod (pi/2) sin(pi x_i); no params; integral 1
"""

GAUSSIAN = r"""
__device__ vegas_real vegas_integrand(const vegas_real* x, int dim, const double* p)
{
    const double a = p[0];
    double s = 0.0;
    for (int i = 0; i < dim; ++i) {
        const double u = x[i] - p[1 + i];
        s += u * u;
    }
    return vegas_real(pow(a * 1.7724538509055160273, -double(dim)) * exp(-s / (a * a)));
}
"""

OSCILLATORY = r"""
__device__ vegas_real vegas_integrand(const vegas_real* x, int dim, const double* p)
{
    double s = 6.283185307179586477 * p[0];
    for (int i = 0; i < dim; ++i) s += p[1 + i] * x[i];
    return vegas_real(cos(s));
}
"""

SINE_PRODUCT = r"""
__device__ vegas_real vegas_integrand(const vegas_real* x, int dim, const double* p)
{
    double f = 1.0;
    for (int i = 0; i < VEGAS_DIM; ++i) f *= 1.5707963267948966192 * sin(3.14159265358979323846 * x[i]);
    return vegas_real(f);
}
"""
