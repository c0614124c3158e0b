// ocml_price.hip -- one kernel per library function used by the integrands (binary64),
// each applied once to every element of an array of arguments drawn from the range the
// integrands pass it.  Run under rocprofv3 --pmc SQ_INSTS_VALU_FLOPS_FP64, the counter
// of each kernel divided by the elements (x 64 lanes per wave) prices one call of the
// function in FP64 FLOPs (add, mul, transcendental instruction = 1, fma = 2), after the
// FLOPs of the identity kernel (loads, stores, none) are subtracted.  Measurement tooling
// for the work per event quoted beside the benchmark; not part of the library.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#define PRICE_KERNEL(name, expr)                                        \
  __global__ void name(const double* __restrict__ a, double* __restrict__ o, int n) { \
    const int i = blockIdx.x * blockDim.x + threadIdx.x;                   \
    if (i < n) {                                                           \
      const double x = a[i];                                               \
      o[i] = (expr);                                                       \
    }                                                                      \
  }

PRICE_KERNEL(k_identity, x)
PRICE_KERNEL(k_atan, atan(x))
PRICE_KERNEL(k_log, log(x))
PRICE_KERNEL(k_exp, exp(x))
PRICE_KERNEL(k_expm1, expm1(x))
PRICE_KERNEL(k_tan, tan(x))
PRICE_KERNEL(k_sqrt, sqrt(x))
PRICE_KERNEL(k_div, 1.0 / x)

// the sine and cosine of one angle (both stored: the second half of o)
__global__ void k_sincos(const double* __restrict__ a, double* __restrict__ o, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    double s, c;
    sincos(a[i], &s, &c);
    o[i] = s;
    o[n + i] = c;
  }
}

int main() {
  const int n = 1 << 22;
  // arguments in the integrands' ranges: atan of (m^2 - M^2)/(M G) for masses from 0 to
  // sqrt(shat) (about -40 .. 1500), log of tau = m^2 / S (1e-9 .. 1), exp of ln tau,
  // expm1 of x ln tau (-20 .. 0), tan on (-pi/2, pi/2), sqrt and reciprocal of (0.1, 1e4),
  // sincos of an azimuth on [0, 2 pi)
  struct Case { const char* name; void (*k)(const double*, double*, int); double lo, hi; bool logscale; };
  const Case cases[] = {{"identity", k_identity, 0.1, 10.0, false}, {"atan", k_atan, -40.0, 1500.0, false},
                        {"log", k_log, 1e-9, 1.0, true},            {"exp", k_exp, -20.0, 0.0, false},
                        {"expm1", k_expm1, -20.0, 0.0, false},      {"tan", k_tan, -1.5, 1.5, false},
                        {"sqrt", k_sqrt, 0.1, 1e4, true},           {"div", k_div, 0.1, 1e4, true},
                        {"sincos", k_sincos, 0.0, 6.283185307179586, false}};
  std::vector<double> h(n);
  double *a = nullptr, *o = nullptr;
  if (hipMalloc(&a, sizeof(double) * n) != hipSuccess || hipMalloc(&o, 2 * sizeof(double) * n) != hipSuccess)
    return 1;
  for (const Case& c : cases) {
    for (int i = 0; i < n; ++i) {
      const double t = (i + 0.5) / n;
      h[i] = c.logscale ? c.lo * std::pow(c.hi / c.lo, t) : c.lo + (c.hi - c.lo) * t;
    }
    if (hipMemcpy(a, h.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess) return 1;
    hipLaunchKernelGGL(c.k, dim3(n / 256), dim3(256), 0, 0, a, o, n);
    if (hipDeviceSynchronize() != hipSuccess) return 1;
    std::printf("%s %d\n", c.name, n);
  }
  (void)hipFree(a);
  (void)hipFree(o);
  return 0;
}
