// FE free step and FE final update, one element / node / ring node at a time,
// as device functions: the FE kernels run them over their grids, and the
// final-update link launches run them as extra workgroups beside the link
// problem (the two are independent, so a launch boundary is saved).
#pragma once

#include "internal.h"

namespace mts {

struct FeTables {
  double N[8][8];       // [gauss point][local node]
  double dN[8][8][3];   // physical derivatives
  double D[6][6];
  double detJ;
};

// Predictor of the FE free problem (beta = 0), one dof: prescribed-velocity
// dofs move at vbc.
__device__ __forceinline__ double fe_predict(const uint8_t *bc, const double *u, const double *v, const double *a,
                                             int64_t t, double dt, double hdt2, double vbc) {
  return bc[t] ? u[t] + dt * vbc : (u[t] + dt * v[t]) + hdt2 * a[t];
}

struct FeElemArgs {
  int64_t ne;
  const int32_t *conn;
  const uint8_t *eact;
  const double *gpa;
  const double *u, *v, *acc;  // v, acc, bc: only with the predictor
  const uint8_t *bc;
  double dt, hdt2, vbc, thick;
  const FeTables *tab;
  double *fe_buf;
};

// Element force f_e = sum_gp alpha B^T D B u_e detJ t (engineering shear strains).
// PRED: u_e is the free problem's predictor of (u, v, a), formed per element
// (the node-wise pass that follows stores the same values).
template <int DIM, bool PRED>
__device__ inline void fe_elem_force_one(const FeElemArgs &E, int64_t e) {
  constexpr int NEN = DIM == 2 ? 4 : 8;
  constexpr int NSTR = DIM == 2 ? 3 : 6;
  if (e >= E.ne || !E.eact[e]) return;
  const FeTables *__restrict__ tab = E.tab;
  double ue[NEN * DIM], fe[NEN * DIM];
  for (int a = 0; a < NEN; a++)
    for (int d = 0; d < DIM; d++) {
      const int64_t t = (int64_t)E.conn[e * NEN + a] * DIM + d;
      if constexpr (PRED) ue[a * DIM + d] = fe_predict(E.bc, E.u, E.v, E.acc, t, E.dt, E.hdt2, E.vbc);
      else ue[a * DIM + d] = E.u[t];
    }
  for (int t = 0; t < NEN * DIM; t++) fe[t] = 0.0;
  for (int g = 0; g < NEN; g++) {
    double al = E.gpa[e * NEN + g];
    if (al == 0.0) continue;
    double eps[NSTR], sig[NSTR];
    for (int r = 0; r < NSTR; r++) eps[r] = 0.0;
    for (int a = 0; a < NEN; a++) {
      const double *dN = tab->dN[g][a];
      const double *uu = ue + a * DIM;
      if (DIM == 2) {
        eps[0] += dN[0] * uu[0];
        eps[1] += dN[1] * uu[1];
        eps[2] += dN[1] * uu[0] + dN[0] * uu[1];
      } else {
        eps[0] += dN[0] * uu[0];
        eps[1] += dN[1] * uu[1];
        eps[2] += dN[2] * uu[2];
        eps[3] += dN[1] * uu[0] + dN[0] * uu[1];
        eps[4] += dN[2] * uu[1] + dN[1] * uu[2];
        eps[5] += dN[2] * uu[0] + dN[0] * uu[2];
      }
    }
    for (int r = 0; r < NSTR; r++) {
      sig[r] = 0.0;
      for (int c = 0; c < NSTR; c++) sig[r] += tab->D[r][c] * eps[c];
    }
    double scale = al * tab->detJ * E.thick;
    for (int a = 0; a < NEN; a++) {
      const double *dN = tab->dN[g][a];
      double *f = fe + a * DIM;
      if (DIM == 2) {
        f[0] += scale * (dN[0] * sig[0] + dN[1] * sig[2]);
        f[1] += scale * (dN[1] * sig[1] + dN[0] * sig[2]);
      } else {
        f[0] += scale * (dN[0] * sig[0] + dN[1] * sig[3] + dN[2] * sig[5]);
        f[1] += scale * (dN[1] * sig[1] + dN[0] * sig[3] + dN[2] * sig[4]);
        f[2] += scale * (dN[2] * sig[2] + dN[1] * sig[4] + dN[0] * sig[5]);
      }
    }
  }
  for (int t = 0; t < NEN * DIM; t++) E.fe_buf[e * NEN * DIM + t] = fe[t];
}

struct FeGatherArgs {
  int64_t nfe;
  int dim, nen;
  const int32_t *n2e_ptr, *n2e;
  const uint8_t *eact, *nact, *bc;
  const double *fe_buf, *PF, *mF;
  double *v, *a;
  double dt, hdt2, hdt, vbc;
  double *at, *vt;
  const int32_t *f2c_ptr;
  double *ut, *u;
};

// Gather element forces per node (ascending element order), then the free
// problem's predictor, acceleration and velocity (Eq. 47a).
// Nodes that carry no multiplier (no constraint interpolates from them) are
// final after the free problem and are written to the state directly.
__device__ inline void fe_gather_free_one(const FeGatherArgs &G, int64_t n) {
  if (n >= G.nfe || !G.nact[n]) return;
  const int dim = G.dim, nen = G.nen;
  double f[3] = {0.0, 0.0, 0.0};
  for (int t = G.n2e_ptr[n]; t < G.n2e_ptr[n + 1]; t++) {
    int64_t e = G.n2e[t] / nen;
    int la = G.n2e[t] % nen;
    if (!G.eact[e]) continue;
    for (int d = 0; d < dim; d++) f[d] += G.fe_buf[(e * nen + la) * dim + d];
  }
  const bool final_now = !G.f2c_ptr || G.f2c_ptr[n + 1] == G.f2c_ptr[n];
  for (int d = 0; d < dim; d++) {
    int64_t t = n * dim + d;
    const double un = fe_predict(G.bc, G.u, G.v, G.a, t, G.dt, G.hdt2, G.vbc);  // as the element pass formed it
    double an, vn;
    if (G.bc[t]) {
      an = 0.0;
      vn = G.vbc;
    } else {
      an = (G.PF[t] - f[d]) / G.mF[n];
      vn = G.v[t] + G.hdt * (G.a[t] + an);
    }
    if (final_now) {
      G.u[t] = un;
      G.v[t] = vn;
      G.a[t] = an;
    } else {
      G.ut[t] = un;
      G.at[t] = an;
      G.vt[t] = vn;
    }
  }
}

struct FeRingArgs {
  int64_t n_ring;
  const int32_t *ring;
  int dim, nen;
  const uint8_t *bc;
  const int32_t *f2c_ptr, *f2c;
  const double *cw, *lam, *mF, *ut, *vt, *at;
  double hdt;
  double *uF, *vF, *aF;
};

// Final update of the overlap FE nodes: U = V + Y^FE lambda with
// Y^FE = (-M^-1 G_F^T, -dt/2 M^-1 G_F^T, 0) (Eq. 50, link problem Eq. 47b at
// beta = 0).  One wavefront per ring node w, lanes over its constraint entries
// (w is uniform per wavefront).
__device__ inline void fe_correct_ring_wave(const FeRingArgs &R, int64_t w, int lane) {
  if (w >= R.n_ring) return;
  const int dim = R.dim, nen = R.nen;
  const int64_t n = R.ring[w];
  double tl[3] = {0.0, 0.0, 0.0};
  for (int t = R.f2c_ptr[n] + lane; t < R.f2c_ptr[n + 1]; t += WAVE) {
    const int64_t q = R.f2c[t] / nen;
    const int aa = R.f2c[t] % nen;
    const double wgt = R.cw[q * nen + aa];
    for (int d = 0; d < dim; d++) tl[d] += wgt * R.lam[q * dim + d];
  }
  for (int off = WAVE / 2; off >= 1; off >>= 1)
    for (int d = 0; d < 3; d++) tl[d] += __shfl_down(tl[d], off, WAVE);
  if (lane != 0) return;
  for (int d = 0; d < dim; d++) {
    const int64_t t = n * dim + d;
    R.uF[t] = R.ut[t];
    if (R.bc[t]) {
      R.vF[t] = R.vt[t];
      R.aF[t] = R.at[t];
    } else {
      const double g = tl[d] / R.mF[n];
      R.aF[t] = R.at[t] - g;
      R.vF[t] = R.vt[t] - R.hdt * g;
    }
  }
}

// Arguments of the three passes for a solver (host side).
FeElemArgs fe_elem_args(Solver &s, bool predict);
FeGatherArgs fe_gather_args(Solver &s);
FeRingArgs fe_ring_args(Solver &s);

}  // namespace mts
