// precompute.h -- host-side construction of the quadrature, the polynomial
// basis and the per-lattice constant tables.
#pragma once
#include <string>
#include <vector>

#include "rlbm_defs.h"

namespace rlbm {

struct QuadHost {
  int d = 0, order = 0, kind = 0, Q = 0, nshell = 0, ndir = 0;
  double m = 0.0;
  double v0 = 0.0;            // massive on-lattice rules: the lattice-speed parameter
  std::vector<int> gfirst;    // massive on-lattice rules: first population of each non-rest group
  std::vector<double> p;      // [Q][d+1]
  std::vector<double> w;      // [Q]
  std::vector<double> disp;   // [Q][d]
};

// Returns 0 on success, else a rlbm_status code with a message in err.
// v0: massive on-lattice rules only (0 = the middle of the admissible window).
int build_quadrature(int d, double m, int order, int kind, double v0, QuadHost &q, std::string &err);

// Massive on-lattice (d+1)-dimensional rules (Sec. 5.3): the v0 window where
// every group weight is >= 0, and the rule at v0 (v0 = 0: the middle of the window).
int massive_window(int d, double m, int order, double &lo, double &hi, std::string &err);
int build_massive(int d, double m, int order, double v0, QuadHost &q, std::string &err);

// Fills the stencil-independent part of the tables (projection rows, moment
// weights, interpolation weights, reference state) for quadrature q.
int build_tables(const QuadHost &q, double tau, double n_ref, int storage, const int64_t extent[3],
                 const int bc[3], Tables &t, std::string &err);

// d = 3: piecewise Chebyshev fits of r(z) = K1(z)/K2(z) in log z and of the
// inverse equation of state, for temperatures T in [kEosTmin, kEosTmax]
// (z = m/T), used by the kernels' equation of state.
int build_eos_fit(double m, Tables &t, std::string &err);

// Rest-frame Maxwell-Juettner moments of the basis monomials (T = 1, U = 0,
// density n): used for the F32_DEV reference and by the kernels' tests.
void basis_moments_host(int d, int order, double m, double n, double T, const double *U, double *M);

}  // namespace rlbm
