// Finite-difference building blocks shared by the acoustic and VTI oracles
// (test infrastructure only; see oracle.h): the 8th-order Fornberg (1988)
// central weights, a zero-padded 2-D grid, and the four 1-D derivatives.
#ifndef SWEEP_ORACLE_STENCIL_H
#define SWEEP_ORACLE_STENCIL_H

#include <omp.h>

#include <cstddef>
#include <vector>

#include "oracle.h"

namespace orc {

// Central-difference weights of Fornberg (1988), 8th order.
// Second derivative: the centre weight -205/72 equals -2 (a1+a2+a3+a4), which is
// what lets the stencil be written in the centred-difference form used below.
inline const double kA2[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
// First derivative: b1..b4 (antisymmetric).
inline const double kA1[5] = {0.0, 4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};

struct Grid2 {
  int NX = 0, NZ = 0;
  size_t size() const { return (size_t)NX * NZ; }
  size_t idx(int i, int j) const { return (size_t)j * NX + i; }
};

typedef std::vector<double> Arr;

// Field value with zero (Dirichlet) outside the padded grid.
inline double val(const Arr& f, const Grid2& g, int i, int j) {
  if (i < 0 || i >= g.NX || j < 0 || j >= g.NZ) return 0.0;
  return f[g.idx(i, j)];
}

// D2x f = sum_k a_k [(f_{i+k} - f_i) + (f_{i-k} - f_i)] / h^2
inline double d2x(const Arr& f, const Grid2& g, int i, int j, double h) {
  const double c = val(f, g, i, j);
  double s = 0.0;
  for (int k = 1; k <= 4; ++k) s += kA2[k] * ((val(f, g, i + k, j) - c) + (val(f, g, i - k, j) - c));
  return s / (h * h);
}
inline double d2z(const Arr& f, const Grid2& g, int i, int j, double h) {
  const double c = val(f, g, i, j);
  double s = 0.0;
  for (int k = 1; k <= 4; ++k) s += kA2[k] * ((val(f, g, i, j + k) - c) + (val(f, g, i, j - k) - c));
  return s / (h * h);
}
// D1x f = sum_k b_k (f_{i+k} - f_{i-k}) / h
inline double d1x(const Arr& f, const Grid2& g, int i, int j, double h) {
  double s = 0.0;
  for (int k = 1; k <= 4; ++k) s += kA1[k] * (val(f, g, i + k, j) - val(f, g, i - k, j));
  return s / h;
}
inline double d1z(const Arr& f, const Grid2& g, int i, int j, double h) {
  double s = 0.0;
  for (int k = 1; k <= 4; ++k) s += kA1[k] * (val(f, g, i, j + k) - val(f, g, i, j - k));
  return s / h;
}

inline int default_threads(const orc_problem* pb) {
  return pb->nthreads > 0 ? pb->nthreads : omp_get_max_threads();
}

}  // namespace orc

#endif
