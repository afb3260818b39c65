// Dalitz-plot membership, one definition for the host runtime (upload
// validation, hf_dalitz_inside) and the device (normalisation grid,
// accept-reject toys), so that a point within rounding of the boundary is
// inside or outside everywhere alike.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace hf {

// Membership of (s_1x, s_1y) with x the partner of particle 1 and y the
// bachelor: s_1x within [(m1+mx)^2, (M-my)^2] and s_1y within the three-body
// limits of s_1y at that s_1x (inclusive).  Evaluated without contractions
// (every product and sum rounded as written) and with correctly rounded
// division and square roots, so host and device give the same answer.
__host__ __device__ inline bool dp_pair_in(double M, double m1, double s1x, double s1y, double mx, double my) {
#pragma clang fp contract(off)
  const double lo = (m1 + mx) * (m1 + mx), hi = (M - my) * (M - my);
  if (!(s1x >= lo && s1x <= hi)) return false;
  const double rs = std::sqrt(s1x);
  const double E1 = (s1x - mx * mx + m1 * m1) / (2.0 * rs);
  const double Ey = (M * M - s1x - my * my) / (2.0 * rs);
  const double p1 = std::sqrt(std::fmax(E1 * E1 - m1 * m1, 0.0));
  const double py = std::sqrt(std::fmax(Ey * Ey - my * my, 0.0));
  const double e = E1 + Ey;
  const double smin = e * e - (p1 + py) * (p1 + py);
  const double smax = e * e - (p1 - py) * (p1 - py);
  return s1y >= smin && s1y <= smax;
}

// A point is inside when both orderings agree (the accepted set is exactly
// symmetric under s12 <-> s13 when m2 = m3).
__host__ __device__ inline bool dp_inside(double M, double m1, double m2, double m3, double s12, double s13) {
  return dp_pair_in(M, m1, s12, s13, m2, m3) && dp_pair_in(M, m1, s13, s12, m3, m2);
}

}  // namespace hf
