// Host FP64 cosmology (no HIP dependency).
#pragma once

namespace cube {

struct Cosmo {
  double om = 1.0, ol = 0.0, ok = 0.0, h = 0.7, sigma8 = 0.8, ns = 1.0;
  double d_norm = 1.0, amp = 1.0;
  double E(double a) const;
  double growth_unnorm(double a) const;
  double D(double a) const { return growth_unnorm(a) / d_norm; }
  double f(double a) const;
  double kick(double a0, double a1) const;
  double drift(double a0, double a1) const;
  double transfer(double k) const;
  double pk(double k, double a) const;  // linear P(k) at a, (Mpc/h)^3
  double pk_shape(double k) const;      // A k^ns T^2(k), i.e. P(k) at a = 1
  void init();
};

}  // namespace cube
