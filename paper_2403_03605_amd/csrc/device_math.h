// Device helpers shared by the kernels of this library.
#pragma once

#include "internal.h"

namespace mts {

// Micromodulus c(|xi|) of Eq. 2: PMB-equivalent c0 / r^3 or exponential c0 exp(-r/l).
__device__ inline double cfun(const Params &P, double r) {
  if (P.kernel == MTS_K_EXP) return P.c0 * exp(-r / P.lexp);
  return P.c0 / (r * r * r);
}

// Arlequin weight alpha(x): cubic / linear / constant in the L-infinity
// distance l1 to the PD-only box, 1 beyond the overlap width (Sec. 3.2).
__device__ inline double alpha_of(const Params &P, const double *xp) {
  if (!P.coupled) return 0.0;
  double l1 = 0.0;
  for (int a = 0; a < P.dim; a++) {
    double d = P.o2lo[a] - xp[a];
    double e = xp[a] - P.o2hi[a];
    if (e > d) d = e;
    if (d > l1) l1 = d;
  }
  if (l1 >= P.overlap) return 1.0;
  if (l1 <= 0.0) return 0.0;
  double t = l1 / P.overlap;
  if (P.weight_kind == MTS_W_LINEAR) return t;
  if (P.weight_kind == MTS_W_CONSTANT) return 0.5;
  return t * t * t;
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Renumber them so that XCD x runs one contiguous range of tiles: the
// neighbour gathers of a tile then hit the L2 that already holds the tiles next
// to it.  A bijection of [0, nb) for any nb.
constexpr int kXcds = 8;
__device__ inline int xcd_block(int b, int nb) {
  const int x = b % kXcds, q = b / kXcds;
  const int base = nb / kXcds, rem = nb % kXcds;
  return x * base + (x < rem ? x : rem) + q;
}

// Position of slot k of local row j in a sliced-ELL slice with L lanes per row.
__device__ inline int64_t sell_slot(int64_t slot_off, int j, int k, int L) {
  return slot_off + (int64_t)(k / L) * WAVE + j * L + (k % L);
}

// Bond state of slot k of row r in the full-lattice layout.
__device__ inline bool full_bit(const int64_t *word_off, const uint64_t *mask, int L, int64_t r, int k) {
  const int S = WAVE / L;
  const int64_t s = r / S;
  const int j = (int)(r % S);
  return (mask[word_off[s] + k / L] >> (j * L + (k % L))) & 1ull;
}

// Exact critical-stretch decision of Eq. 3-4, s = (|xi+eta| - |xi|)/|xi| >= s_crit,
// evaluated without square roots except in a narrow band around the threshold:
// outside |y2 / ((1+s_crit)^2 r2) - 1| <= 1e-12 the sign of the decision is
// certain (rounding of the plain formula is below 1e-15 relative), inside it the
// plain formula decides, so the outcome always equals the plain formula's.
__device__ inline bool breaks(double r2, double y2, double K2, double scrit) {
  const double thr = K2 * r2;
  if (y2 <= thr * (1.0 - 1e-12)) return false;
  if (y2 >= thr * (1.0 + 1e-12)) return true;
  const double r = sqrt(r2), ly = sqrt(y2);
  return (ly - r) / r >= scrit;
}

}  // namespace mts
