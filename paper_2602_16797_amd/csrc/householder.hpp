// Householder reflector coefficients shared by the QR panels and TSQR.
#pragma once
#include "common.hpp"

namespace rl {

// Householder coefficients for a real beta with |beta| = |(alpha, x)| and the
// sign opposite to re(alpha): tau = (beta - alpha) / beta and
// sc = 1 / (alpha - beta), the scale of the reflector's tail.  For complex
// alpha the quotient by alpha - beta = z takes one real reciprocal,
// conj(z) / |z|^2, where |z|^2 is representable (|re z| = |re alpha| + |beta|
// bounds |z| within a factor sqrt(2)), else Smith's quotient.
__device__ inline void hh_coef(double alpha, double beta, double& tau, double& sc) {
  tau = (beta - alpha) / beta;
  sc = 1.0 / (alpha - beta);
}
__device__ inline void hh_coef(cd alpha, double beta, cd& tau, cd& sc) {
  const double ib = 1.0 / beta;
  tau = cd{(beta - alpha.x) * ib, -alpha.y * ib};
  const double zx = alpha.x - beta, zy = alpha.y;
  const double az = fabs(zx);
  if (az > 1e-140 && az < 1e140) {
    const double iz = 1.0 / (zx * zx + zy * zy);
    sc = cd{zx * iz, -zy * iz};
  } else {
    sc = divs(cd{1.0, 0.0}, cd{zx, zy});
  }
}
__device__ inline void hh_coef(float alpha, double beta, float& tau, float& sc) {
  const float b = (float)beta;
  tau = (b - alpha) / b;
  sc = 1.0f / (alpha - b);
}

}  // namespace rl
