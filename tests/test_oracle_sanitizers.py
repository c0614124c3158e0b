"""The oracle under the host sanitizers (CPU only): compiled with gcc's
AddressSanitizer and UndefinedBehaviorSanitizer, a small C driver runs every
process, the observable histogram, equal-count and adaptive stratification (with
injected counts), the adjoint, grid injection and teardown; any out-of-bounds
access, leak or undefined operation fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
#include "vegas_oracle.h"

static void phys(double *p, double sqrts, double mlo, double mhi, double ptmin, double etamax) {
  const double v[ORA_NPHYS] = {1.0 / 128.0, 0.2224, 91.1876, 2.4952, 80.4, 2.1, 0, 1.0, -0.5, 3.0,
                               0, 0, 0, 0, 1.0, 0.3893794e9};
  for (int k = 0; k < ORA_NPHYS; ++k) p[k] = v[k];
  p[ORA_P_SQRTS] = sqrts; p[ORA_P_MLO] = mlo; p[ORA_P_MHI] = mhi;
  p[ORA_P_PTMIN] = ptmin; p[ORA_P_ETAMAX] = etamax;
}

static int run(int process, int ndim, const double *par, int np, int strata, double beta, int nobs,
               double lo, double hi) {
  ora_state *s = ora_create(process, ndim, 20, 3, 1.5, par, np);
  if (!s) return 1;
  int D = ora_ndim(process, ndim);
  if (strata && ora_set_strata(s, strata)) return 2;
  if (beta > 0 && ora_set_strata_beta(s, beta)) return 3;
  if (nobs && ora_set_observable(s, nobs, lo, hi, 1)) return 4;
  double out[4];
  for (int it = 0; it < 3; ++it) {
    if (ora_iterate(s, 3001, out)) return 5;
    if (ora_refine(s)) return 6;
  }
  if (beta > 0) {
    int64_t H = ora_strata_cubes(s);
    int64_t *c = (int64_t *)malloc(sizeof(int64_t) * (size_t)H);
    if (ora_strata_next_counts(s, 3001, c)) return 7;
    if (ora_inject_strata_counts(s, c)) return 8;
    if (ora_iterate(s, 3001, out)) return 9;
    if (ora_get_strata_counts(s, c)) return 10;
    free(c);
  }
  if (nobs) {
    double *a = (double *)malloc(sizeof(double) * (size_t)(4 * (nobs + 2)));
    if (ora_get_observable(s, a, a + nobs + 2, a + 2 * (nobs + 2), a + 3 * (nobs + 2))) return 11;
    free(a);
  }
  double *e = (double *)malloc(sizeof(double) * (size_t)(D * 21));
  ora_get_grid(s, e);
  ora_set_grid(s, e);
  double *w = (double *)malloc(sizeof(double) * 50);
  unsigned char *b = (unsigned char *)malloc((size_t)(50 * D));
  ora_event_weights(s, 0, 0, 50, w, b);
  double r[4];
  if (ora_result_from(s, 1, r)) return 12;
  free(e); free(w); free(b);
  ora_destroy(s);
  return 0;
}

int main(void) {
  double g[2] = {0.5, 0.2}, p[ORA_NPHYS];
  int rc = 0;
  rc |= run(ORA_GAUSS, 4, g, 2, 0, 0.0, 7, 0.2, 0.8);
  rc |= run(ORA_GAUSS, 3, g, 2, 3, 0.0, 0, 0, 0);
  rc |= run(ORA_GAUSS, 3, g, 2, 3, 0.75, 5, 0.1, 0.9);
  phys(p, 91.0, 0, 0, 0, 1e300);   rc |= run(ORA_EEMUMU, 0, p, ORA_NPHYS, 4, 0.0, 8, -1, 1);
  phys(p, 13000, 81, 101, 0, 1e300); rc |= run(ORA_DY_Z, 0, p, ORA_NPHYS, 0, 0.0, 10, 81, 101);
  phys(p, 13000, 40, 0, 20, 2.5);  rc |= run(ORA_W_PLUS, 0, p, ORA_NPHYS, 3, 1.0, 12, 20, 70);
  phys(p, 500, 0, 0, 0, 1e300);    rc |= run(ORA_WW_4L, 0, p, ORA_NPHYS, 0, 0.0, 6, 60, 100);
  phys(p, 13000, 150, 0, 0, 1e300); rc |= run(ORA_WW_HAD, 0, p, ORA_NPHYS, 0, 0.0, 6, 60, 100);
  phys(p, 13000, 81, 101, 0, 1e300);
  {
    ora_state *s = ora_create(ORA_DY_Z, 0, 20, 1, 1.5, p, ORA_NPHYS);
    double th[5] = {91.1876, 2.4952, 0.2224, -0.5, 3.0}, sig, ds[5];
    rc |= ora_dy_grad(s, 0, 500, th, &sig, ds) != 0;
    ora_destroy(s);
  }
  printf("driver rc %d\n", rc);
  return rc;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "vegas_oracle.c"),
           str(drv), "-lm", "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "driver rc 0" in r.stdout
