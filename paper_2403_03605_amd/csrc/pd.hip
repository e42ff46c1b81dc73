// Peridynamic subdomain on the device: Arlequin weights and masses, the fused
// substep kernel (bond stretch, irreversible breaking, pairwise force, velocity
// Verlet corrector and the next predictor), the link-problem substep used for
// the unit-load responses and for the final update, and nodal damage.
//
// Equations: Eq. 2 (force), Eq. 3 (stretch), Eq. 4 (bond state), Eq. 5 (damage),
// Eq. 38 with gamma = 1/2, beta = 0 (velocity Verlet), Eq. 48a/48b (free and
// link problems), Eq. 17-18 and Eq. 34 (Arlequin weights of stiffness and mass).
#include "internal.h"

namespace mts {

namespace {

constexpr int kBlock = 256;  // 4 wavefronts = 4 slices per workgroup

__device__ inline double cfun(const Params &P, double r) {
  if (P.kernel == MTS_K_EXP) return P.c0 * exp(-r / P.lexp);
  return P.c0 / (r * r * r);
}

// alpha(x): cubic / linear / constant in the L-infinity distance l1 to the
// PD-only box Omega^2, 1 beyond the overlap width (Sec. 3.2 weight functions).
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

__global__ void k_alpha_mass(Params P, const double *x, int64_t N, double *alpha, double *mass) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double xp[3] = {x[i], x[N + i], P.dim == 3 ? x[2 * N + i] : 0.0};
  double al = alpha_of(P, xp);
  alpha[i] = al;
  mass[i] = (1.0 - al) * P.rho * P.V;
}

// Pure-PD loading: traction as a body force traction/delta within delta of the y faces.
__global__ void k_body_force(Params P, const double *x, int64_t N, double lo_y, double hi_y, double T,
                             double *Pf) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double y = x[N + i];
  double b = 0.0;
  if (y - lo_y < P.delta) b = -T / P.delta * P.V;
  else if (hi_y - y < P.delta) b = T / P.delta * P.V;
  Pf[i] = 0.0;
  Pf[N + i] = b;
  if (P.dim == 3) Pf[2 * N + i] = 0.0;
}

__global__ void k_init_accel(int64_t N, int dim, const double *Pf, const double *mass, double *a) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  for (int d = 0; d < dim; d++) a[d * N + i] = (Pf ? Pf[d * N + i] : 0.0) / mass[i];
}

__global__ void k_predict(int64_t N, int dim, double dt, double hdt2, const double *u, const double *v,
                          const double *a, double *up) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  for (int d = 0; d < dim; d++) {
    int64_t t = d * N + i;
    up[t] = (u[t] + dt * v[t]) + hdt2 * a[t];
  }
}

struct SubstepArgs {
  const double *x;
  int64_t N, n_slices;
  const int32_t *width;
  const int64_t *slot_off, *word_off;
  const int32_t *col;
  uint64_t *mask;
  const double *alpha, *mass, *P;
  const double *u_in;   // u_j (predicted)
  double *u_out;        // u_{j+1} predicted
  double *v, *a;
  const int32_t *cidx;
  const double *lam0;
  double sfac;
  const uint8_t *in_region;
  int32_t *region_flag;
  const int32_t *rp;
  double *damage;       // written when non-null
  int breaking;
};

// One lane = one PD node, one wavefront = one slice of 64 consecutive nodes.
// The lane sums its own family in canonical order (no atomics); bond states of
// the slice's slot k form one 64-bit word owned by the wavefront.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_pd_substep(SubstepArgs A, Params P) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t slice = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  if (slice >= A.n_slices) return;  // uniform per wavefront
  const int64_t N = A.N;
  const int64_t i = slice * WAVE + lane;
  const bool valid = i < N;
  const int64_t ii = valid ? i : 0;
  const int w = A.width[slice];
  const int64_t so = A.slot_off[slice], wo = A.word_off[slice];
  double xi_[3], ui_[3];
  for (int d = 0; d < DIM; d++) {
    xi_[d] = A.x[d * N + ii];
    ui_[d] = A.u_in[d * N + ii];
  }
  const double al_i = A.alpha[ii];
  double F[3] = {0.0, 0.0, 0.0};
  int n_intact = 0;
  bool broke = false;
  for (int k = 0; k < w; k++) {
    const uint64_t word = A.mask[wo + k];
    bool bit = (word >> lane) & 1ull;
    if (bit) {
      const int64_t c = A.col[so + (int64_t)k * WAVE + lane];
      double xi[3], eta[3];
      for (int d = 0; d < DIM; d++) {
        xi[d] = A.x[d * N + c] - xi_[d];
        eta[d] = A.u_in[d * N + c] - ui_[d];
      }
      double r2 = xi[0] * xi[0] + xi[1] * xi[1];
      if (DIM == 3) r2 = r2 + xi[2] * xi[2];
      const double r = sqrt(r2);
      if (A.breaking) {
        double y[3];
        for (int d = 0; d < DIM; d++) y[d] = xi[d] + eta[d];
        double y2 = y[0] * y[0] + y[1] * y[1];
        if (DIM == 3) y2 = y2 + y[2] * y[2];
        const double ly = sqrt(y2);
        const double st = (ly - r) / r;  // Eq. 3
        if (st >= P.scrit) {             // Eq. 4, inclusive
          bit = false;
          broke = true;
        }
      }
      if (bit) {
        double xe = xi[0] * eta[0] + xi[1] * eta[1];
        if (DIM == 3) xe = xe + xi[2] * eta[2];
        const double wgt = 1.0 - 0.5 * (al_i + A.alpha[c]);
        const double tt = ((wgt * cfun(P, r)) * xe) * P.VV;  // Eq. 2 times V_i V_k
        for (int d = 0; d < DIM; d++) F[d] += tt * xi[d];
        n_intact++;
      }
    }
    const uint64_t nw = __ballot(bit);
    if (nw != word && lane == 0) A.mask[wo + k] = nw;
  }
  if (!valid) return;
  if (broke && A.in_region && A.in_region[i]) A.region_flag[0] = 1;
  const int32_t q = A.cidx ? A.cidx[i] : -1;
  const double m_i = A.mass[i];
  for (int d = 0; d < DIM; d++) {
    const int64_t t = d * N + i;
    double fl = F[d] + (A.P ? A.P[t] : 0.0);
    if (q >= 0) fl = fl + A.sfac * A.lam0[q * DIM + d];  // + G_P^T S_j
    const double an = fl / m_i;
    const double ao = A.a[t];
    const double vn = A.v[t] + P.hdtP * (ao + an);
    A.a[t] = an;
    A.v[t] = vn;
    A.u_out[t] = (ui_[d] + P.dtP * vn) + P.hdt2P * an;
  }
  if (A.damage) {
    const int fam = A.rp[i + 1] - A.rp[i];
    A.damage[i] = fam > 0 ? 1.0 - (double)n_intact / (double)fam : 0.0;
  }
}

// Link problem (Eq. 48b / eq. unit): linear, no breaking, bond states of the
// last rebuild.  NRHS right-hand sides share one pass over the bond data.
//  kColor = false: one RHS, load (j/m) lambda_m at every constraint node.
//  kColor = true : RHS b loads (j/m) e_dir(b) at every constraint node of color(b).
struct LinkArgs {
  const double *x;
  int64_t N, n_rows, n_slices;
  const int32_t *rows, *width;
  const int64_t *slot_off, *word_off;
  const int32_t *col;
  const uint64_t *mask;
  const double *alpha, *mass;
  const double *u_in;
  double *u_out, *v, *a;  // [NRHS][DIM][N]
  const int32_t *cidx;
  const double *lam;      // kColor = false
  const int32_t *ccolor;  // kColor = true: color of each constraint
  int32_t rhs_color[16];
  int32_t rhs_dir[16];
  double lfac;
};

template <int DIM, int NRHS, bool kColor>
__global__ __launch_bounds__(kBlock) void k_link_substep(LinkArgs A, Params P) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t slice = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  if (slice >= A.n_slices) return;
  const int64_t r = slice * WAVE + lane;
  const bool valid = r < A.n_rows;
  const int64_t N = A.N;
  const int64_t i = valid ? A.rows[r] : A.rows[0];
  const int w = A.width[slice];
  const int64_t so = A.slot_off[slice], wo = A.word_off[slice];
  const int64_t stride = (int64_t)DIM * N;
  double xi_[3], ui_[NRHS][3];
  for (int d = 0; d < DIM; d++) xi_[d] = A.x[d * N + i];
  for (int b = 0; b < NRHS; b++)
    for (int d = 0; d < DIM; d++) ui_[b][d] = A.u_in[b * stride + d * N + i];
  const double al_i = A.alpha[i];
  double F[NRHS][3];
  for (int b = 0; b < NRHS; b++) F[b][0] = F[b][1] = F[b][2] = 0.0;
  for (int k = 0; k < w; k++) {
    const uint64_t word = A.mask[wo + k];
    if (!((word >> lane) & 1ull)) continue;
    const int64_t c = A.col[so + (int64_t)k * WAVE + lane];
    double xi[3];
    for (int d = 0; d < DIM; d++) xi[d] = A.x[d * N + c] - xi_[d];
    double r2 = xi[0] * xi[0] + xi[1] * xi[1];
    if (DIM == 3) r2 = r2 + xi[2] * xi[2];
    const double rr = sqrt(r2);
    const double wgt = 1.0 - 0.5 * (al_i + A.alpha[c]);
    const double coef = (wgt * cfun(P, rr));
    for (int b = 0; b < NRHS; b++) {
      double xe = xi[0] * (A.u_in[b * stride + c] - ui_[b][0]) + xi[1] * (A.u_in[b * stride + N + c] - ui_[b][1]);
      if (DIM == 3) xe = xe + xi[2] * (A.u_in[b * stride + 2 * N + c] - ui_[b][2]);
      const double tt = (coef * xe) * P.VV;
      for (int d = 0; d < DIM; d++) F[b][d] += tt * xi[d];
    }
  }
  if (!valid) return;
  const int32_t q = A.cidx[i];
  const double m_i = A.mass[i];
  for (int b = 0; b < NRHS; b++)
    for (int d = 0; d < DIM; d++) {
      const int64_t t = b * stride + d * N + i;
      double fl = F[b][d];
      if (q >= 0) {
        if (kColor) {
          if (A.ccolor[q] == A.rhs_color[b] && d == A.rhs_dir[b]) fl = fl + A.lfac;
        } else {
          fl = fl + A.lfac * A.lam[q * DIM + d];
        }
      }
      const double an = fl / m_i;
      const double vn = A.v[t] + P.hdtP * (A.a[t] + an);
      A.a[t] = an;
      A.v[t] = vn;
      A.u_out[t] = (ui_[b][d] + P.dtP * vn) + P.hdt2P * an;
    }
}

__global__ void k_zero_region(int64_t n_rows, const int32_t *rows, int64_t N, int dim, int nrhs, double *u0,
                              double *u1, double *v, double *a) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rows) return;
  int64_t i = rows[r];
  for (int b = 0; b < nrhs; b++)
    for (int d = 0; d < dim; d++) {
      int64_t t = ((int64_t)b * dim + d) * N + i;
      u0[t] = 0.0;
      u1[t] = 0.0;
      v[t] = 0.0;
      a[t] = 0.0;
    }
}

// U = V + W on the link region, then the predictor for the next substep.
__global__ void k_add_link(int64_t n_rows, const int32_t *rows, int64_t N, int dim, double dt, double hdt2,
                           const double *Wu, const double *Wv, const double *Wa, double *u, double *v, double *a,
                           double *u_pred) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rows) return;
  int64_t i = rows[r];
  for (int d = 0; d < dim; d++) {
    int64_t t = d * N + i;
    double un = u[t] + Wu[t];
    double vn = v[t] + Wv[t];
    double an = a[t] + Wa[t];
    u[t] = un;
    v[t] = vn;
    a[t] = an;
    u_pred[t] = (un + dt * vn) + hdt2 * an;
  }
}

__global__ void k_damage(int64_t N, int64_t n_slices, const int32_t *width, const int64_t *word_off,
                         const uint64_t *mask, const int32_t *rp, double *phi) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int64_t s = i / WAVE;
  int lane = (int)(i % WAVE);
  int cnt = 0;
  for (int k = 0; k < width[s]; k++) cnt += (int)((mask[word_off[s] + k] >> lane) & 1ull);
  int fam = rp[i + 1] - rp[i];
  phi[i] = fam > 0 ? 1.0 - (double)cnt / (double)fam : 0.0;
}

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void pd_setup(Solver &s) {
  const int64_t N = s.N;
  hipStream_t st = s.stream;
  k_alpha_mass<<<nblk(N), 256, 0, st>>>(s.prm, s.x, N, s.alpha, s.mass);
  MTS_LAUNCH_CHECK();
  if (s.p.mode == MTS_PURE_PD && s.p.traction != 0.0) {
    s.P = s.arena.alloc<double>((size_t)s.dim * N);
    k_body_force<<<nblk(N), 256, 0, st>>>(s.prm, s.x, N, s.p.pd_lo[1], s.p.pd_hi[1], s.p.traction, s.P);
    MTS_LAUNCH_CHECK();
  }
  k_init_accel<<<nblk(N), 256, 0, st>>>(N, s.dim, s.P, s.mass, s.a);
  MTS_LAUNCH_CHECK();
}

void pd_predict_all(Solver &s) {
  k_predict<<<nblk(s.N), 256, 0, s.stream>>>(s.N, s.dim, s.prm.dtP, s.prm.hdt2P, s.u[s.cur], s.v, s.a,
                                             s.u[s.cur ^ 1]);
  MTS_LAUNCH_CHECK();
}

// Substep j (1..m) of the free problem.  Reads u[cur^1] (predicted u_j), writes
// the predicted u_{j+1} into u[cur]; afterwards cur flips.
void pd_substep(Solver &s, int j) {
  SubstepArgs A{};
  A.x = s.x;
  A.N = s.N;
  A.n_slices = s.sell.n_slices;
  A.width = s.sell.width;
  A.slot_off = s.sell.slot_off;
  A.word_off = s.sell.word_off;
  A.col = s.sell.col;
  A.mask = s.sell.mask;
  A.alpha = s.alpha;
  A.mass = s.mass;
  A.P = s.P;
  A.u_in = s.u[s.cur ^ 1];
  A.u_out = s.u[s.cur];
  A.v = s.v;
  A.a = s.a;
  A.cidx = s.nc ? s.cidx : nullptr;
  A.lam0 = s.lam0;
  A.sfac = 1.0 - (double)j / (double)s.m;
  A.in_region = s.nc ? s.in_region : nullptr;
  A.region_flag = s.region_flag;
  A.rp = s.rp;
  A.damage = (j == s.m) ? s.damage : nullptr;
  A.breaking = s.breaking ? 1 : 0;
  unsigned grid = (unsigned)((A.n_slices * WAVE + kBlock - 1) / kBlock);
  hipEvent_t e0 = nullptr;
  s.prof_begin(MTS_KT_PD_SUBSTEP, &e0);
  if (s.dim == 2) k_pd_substep<2><<<grid, kBlock, 0, s.stream>>>(A, s.prm);
  else k_pd_substep<3><<<grid, kBlock, 0, s.stream>>>(A, s.prm);
  MTS_LAUNCH_CHECK();
  s.prof_end(MTS_KT_PD_SUBSTEP, e0);
  s.cur ^= 1;
  s.pd_steps++;
}

void pd_damage(Solver &s) {
  k_damage<<<nblk(s.N), 256, 0, s.stream>>>(s.N, s.sell.n_slices, s.sell.width, s.sell.word_off, s.sell.mask,
                                            s.rp, s.damage);
  MTS_LAUNCH_CHECK();
}

// ---- link runs (used by coupling.hip) ----
void link_zero(Solver &s, double *u0, double *u1, double *v, double *a, int nrhs) {
  if (!s.rsell.n_rows) return;
  k_zero_region<<<nblk(s.rsell.n_rows), 256, 0, s.stream>>>(s.rsell.n_rows, s.rsell.rows, s.N, s.dim, nrhs, u0, u1,
                                                            v, a);
  MTS_LAUNCH_CHECK();
}

template <int DIM, int NRHS, bool kColor>
static void launch_link(Solver &s, LinkArgs &A) {
  unsigned grid = (unsigned)((A.n_slices * WAVE + kBlock - 1) / kBlock);
  k_link_substep<DIM, NRHS, kColor><<<grid, kBlock, 0, s.stream>>>(A, s.prm);
  MTS_LAUNCH_CHECK();
}

// One link substep j over the region rows.  u_in/u_out/v/a: [nrhs][dim][N].
void link_substep(Solver &s, int j, const double *u_in, double *u_out, double *v, double *a, const double *lam,
                  const int32_t *ccolor, const int32_t *rhs_color, const int32_t *rhs_dir, int nrhs) {
  if (!s.rsell.n_rows) return;
  LinkArgs A{};
  A.x = s.x;
  A.N = s.N;
  A.n_rows = s.rsell.n_rows;
  A.n_slices = s.rsell.n_slices;
  A.rows = s.rsell.rows;
  A.width = s.rsell.width;
  A.slot_off = s.rsell.slot_off;
  A.word_off = s.rsell.word_off;
  A.col = s.rsell.col;
  A.mask = s.rsell.mask;
  A.alpha = s.alpha;
  A.mass = s.mass;
  A.u_in = u_in;
  A.u_out = u_out;
  A.v = v;
  A.a = a;
  A.cidx = s.cidx;
  A.lam = lam;
  A.ccolor = ccolor;
  for (int b = 0; b < nrhs && rhs_color; b++) {
    A.rhs_color[b] = rhs_color[b];
    A.rhs_dir[b] = rhs_dir[b];
  }
  A.lfac = (double)j / (double)s.m;
  if (!ccolor) {
    if (s.dim == 2) launch_link<2, 1, false>(s, A);
    else launch_link<3, 1, false>(s, A);
  } else if (s.dim == 2) {
    if (nrhs != 8) throw ArgError{"link batch must hold 8 right-hand sides in 2D"};
    launch_link<2, 8, true>(s, A);
  } else {
    if (nrhs != 6) throw ArgError{"link batch must hold 6 right-hand sides in 3D"};
    launch_link<3, 6, true>(s, A);
  }
}

void link_add(Solver &s, const double *Wu, const double *Wv, const double *Wa) {
  if (!s.rsell.n_rows) return;
  k_add_link<<<nblk(s.rsell.n_rows), 256, 0, s.stream>>>(s.rsell.n_rows, s.rsell.rows, s.N, s.dim, s.prm.dtP,
                                                         s.prm.hdt2P, Wu, Wv, Wa, s.u[s.cur], s.v, s.a,
                                                         s.u[s.cur ^ 1]);
  MTS_LAUNCH_CHECK();
}

}  // namespace mts
