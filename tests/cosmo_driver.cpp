// Test-only C wrapper around the library's host cosmology (csrc/cosmo.cpp), built with g++ by
// tests/test_host_cosmology.py to compare it with the oracle on the CPU.
#include "../paper_1712_06121_amd/csrc/cosmo.h"

extern "C" int cosmo_eval(double om, double ol, double h, double s8, double ns, int n, const double* a0,
                          const double* a1, double* kick, double* drift, double* D, double* f, double* amp) {
  cube::Cosmo c;
  c.om = om;
  c.ol = ol;
  c.h = h;
  c.sigma8 = s8;
  c.ns = ns;
  c.init();
  for (int i = 0; i < n; ++i) {
    kick[i] = c.kick(a0[i], a1[i]);
    drift[i] = c.drift(a0[i], a1[i]);
    D[i] = c.D(a1[i]);
    f[i] = c.f(a1[i]);
  }
  *amp = c.amp;
  return 0;
}
