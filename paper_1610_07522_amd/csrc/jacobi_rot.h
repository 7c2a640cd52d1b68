// Complex FP64 helpers and the 2x2 Hermitian Jacobi rotation shared by the
// blocked Jacobi eigensolver and the eigenvector refinement (Sec. 3.3.2).
#pragma once

#include <hip/hip_runtime.h>

namespace sky {
namespace jrot {

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cmulc(double2 a, double2 b) {  // a * conj(b)
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ inline double2 cconjmul(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }

// Rotation of the 2x2 Hermitian [[a, r e^{i phi}], [r e^{-i phi}, b]]:
// G = [[e^{i phi} c, e^{i phi} s], [-s, c]], G^H S G diagonal.
struct Rot {
  double c, s, er, ei;  // cos, sin, e^{i phi}
};

__device__ inline Rot make_rot(double a, double b, double2 apq) {
  Rot g;
  // |a_pq| by a scaled hypot: the plain sqrt(x^2 + y^2) underflows for the
  // ~1e-160 couplings that quadratic convergence produces, which would give
  // |e^{i phi}| != 1 and a non-unitary rotation.  Couplings below 1e-18 of
  // the diagonal scale are treated as converged (no rotation).
  const double r = hypot(apq.x, apq.y);
  if (!(r > 1e-18 * (fabs(a) + fabs(b))) || r < 1e-250) {
    g.c = 1.0; g.s = 0.0; g.er = 1.0; g.ei = 0.0;
    return g;
  }
  g.er = apq.x / r;
  g.ei = apq.y / r;
  double zeta = (b - a) / (2.0 * r);
  double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
  g.c = 1.0 / sqrt(1.0 + t * t);
  g.s = t * g.c;
  return g;
}

// Round-robin partner pairs of round r among np players: pair i -> (p, q).
__device__ inline void rr_pair(int np, int r, int i, int& p, int& q) {
  const int n1 = np - 1;
  p = (i == 0) ? 0 : ((i + r - 1) % n1) + 1;
  q = ((n1 - i + r - 1) % n1) + 1;
}

}  // namespace jrot
}  // namespace sky
