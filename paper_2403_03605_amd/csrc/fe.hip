// Finite-element subdomain on the device: Q4 (2D, plane stress) / Hex8 (3D)
// elements with 2x2(x2) Gauss points, the Arlequin weight alpha evaluated at
// every Gauss point of the stiffness and of the row-sum lumped mass (Eq. 24-34),
// explicit Newmark (gamma = 1/2, beta = 0) at dt_FE = m dt_PD, element forces
// computed per element and gathered per node in a fixed order (no atomics).
#include "fe_device.h"

#include <cmath>

namespace mts {

namespace {

__device__ inline double nat(int dim, int a, int c) {
  // local node a natural coordinate along axis c: Q4 (-1,-1),(1,-1),(1,1),(-1,1); Hex8 adds z.
  const int q4[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};
  if (c == 2) return a < 4 ? -1.0 : 1.0;
  return (double)q4[a & 3][c];
}

__device__ inline double shape_fn(int dim, int a, const double *xi) {
  if (dim == 2) return 0.25 * (1.0 + nat(2, a, 0) * xi[0]) * (1.0 + nat(2, a, 1) * xi[1]);
  return 0.125 * (1.0 + nat(3, a, 0) * xi[0]) * (1.0 + nat(3, a, 1) * xi[1]) * (1.0 + nat(3, a, 2) * xi[2]);
}

__device__ inline void gauss_nat(int dim, int g, double *xi) {
  double q = 1.0 / sqrt(3.0);
  xi[0] = (g & 1) ? q : -q;
  xi[1] = (g & 2) ? q : -q;
  if (dim == 3) xi[2] = (g & 4) ? q : -q;
}

// Shape functions, their derivatives at the Gauss points and Hooke's law (Eq. 9).
__global__ void k_fe_tables(int dim, double h, double E, double nu, FeTables *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  FeTables T{};
  int nen = dim == 2 ? 4 : 8;
  double g2 = 2.0 / h;
  for (int g = 0; g < nen; g++) {
    double xi[3];
    gauss_nat(dim, g, xi);
    for (int a = 0; a < nen; a++) {
      T.N[g][a] = shape_fn(dim, a, xi);
      if (dim == 2) {
        T.dN[g][a][0] = g2 * 0.25 * nat(2, a, 0) * (1.0 + nat(2, a, 1) * xi[1]);
        T.dN[g][a][1] = g2 * 0.25 * nat(2, a, 1) * (1.0 + nat(2, a, 0) * xi[0]);
      } else {
        T.dN[g][a][0] = g2 * 0.125 * nat(3, a, 0) * (1.0 + nat(3, a, 1) * xi[1]) * (1.0 + nat(3, a, 2) * xi[2]);
        T.dN[g][a][1] = g2 * 0.125 * nat(3, a, 1) * (1.0 + nat(3, a, 0) * xi[0]) * (1.0 + nat(3, a, 2) * xi[2]);
        T.dN[g][a][2] = g2 * 0.125 * nat(3, a, 2) * (1.0 + nat(3, a, 0) * xi[0]) * (1.0 + nat(3, a, 1) * xi[1]);
      }
    }
  }
  if (dim == 2) {
    double k = E / (1.0 - nu * nu);
    T.D[0][0] = k;
    T.D[0][1] = k * nu;
    T.D[1][0] = k * nu;
    T.D[1][1] = k;
    T.D[2][2] = k * (1.0 - nu) / 2.0;
    T.detJ = (h / 2) * (h / 2);
  } else {
    double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    double mu = E / (2.0 * (1.0 + nu));
    for (int r = 0; r < 3; r++)
      for (int c = 0; c < 3; c++) T.D[r][c] = lam + (r == c ? 2.0 * mu : 0.0);
    T.D[3][3] = T.D[4][4] = T.D[5][5] = mu;
    T.detJ = (h / 2) * (h / 2) * (h / 2);
  }
  *out = T;
}

__device__ inline double alpha_fe(const Params &P, const double *xp) {
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

struct MeshGeo {
  double lo[3];
  double h;
  int64_t ne[3];
};

__global__ void k_fe_gp_alpha(Params P, MeshGeo G, int64_t ne, int ngp, double *gpa, uint8_t *eact) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  int64_t ex = e % G.ne[0], ey = (e / G.ne[0]) % G.ne[1], ez = e / (G.ne[0] * G.ne[1]);
  double x0[3] = {G.lo[0] + (double)ex * G.h, G.lo[1] + (double)ey * G.h,
                  P.dim == 3 ? G.lo[2] + (double)ez * G.h : 0.0};
  int act = 0;
  for (int g = 0; g < ngp; g++) {
    double xi[3], xg[3];
    gauss_nat(P.dim, g, xi);
    for (int d = 0; d < P.dim; d++) xg[d] = x0[d] + (xi[d] + 1.0) * (G.h / 2.0);
    double al = alpha_fe(P, xg);
    gpa[e * ngp + g] = al;
    if (al > 0.0) act = 1;
  }
  eact[e] = (uint8_t)act;
}

// Per node: lumped weighted mass, traction load, activity.  The node's
// (element, local node) list is in ascending element order.
__global__ void k_fe_node_setup(Params P, MeshGeo G, int64_t nfe, int nen, int ngp, const int32_t *n2e_ptr,
                                const int32_t *n2e, const double *gpa, const uint8_t *eact, double T,
                                double dom_hi_y, double Tx, double dom_hi_x, double thick, double *mF, double *PF,
                                uint8_t *nact, const FeTables *tab) {
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nfe) return;
  int dim = P.dim;
  double m = 0.0, py = 0.0, px = 0.0;
  int act = 0;
  double q = 1.0 / sqrt(3.0);
  for (int t = n2e_ptr[n]; t < n2e_ptr[n + 1]; t++) {
    int64_t e = n2e[t] / nen;
    int a = n2e[t] % nen;
    if (!eact[e]) continue;
    act = 1;
    for (int g = 0; g < ngp; g++) m += gpa[e * ngp + g] * P.rho * tab->N[g][a] * tab->detJ * thick;
  }
  if (T != 0.0) {
    for (int t = n2e_ptr[n]; t < n2e_ptr[n + 1]; t++) {
      int64_t e = n2e[t] / nen;
      int a = n2e[t] % nen;
      if (!eact[e]) continue;
      int64_t ex = e % G.ne[0], ey = (e / G.ne[0]) % G.ne[1], ez = e / (G.ne[0] * G.ne[1]);
      for (int side = 0; side < 2; side++) {
        if ((side == 0 && ey != 0) || (side == 1 && ey != G.ne[1] - 1)) continue;
        double eta = side == 0 ? -1.0 : 1.0;
        double ty = side == 0 ? -T : T;
        int ngp2 = dim == 2 ? 2 : 4;
        for (int g = 0; g < ngp2; g++) {
          double xi[3] = {(g & 1) ? q : -q, eta, (g & 2) ? q : -q};
          double xg[3] = {G.lo[0] + (double)ex * G.h + (xi[0] + 1.0) * (G.h / 2.0), side == 0 ? G.lo[1] : dom_hi_y,
                          dim == 3 ? G.lo[2] + (double)ez * G.h + (xi[2] + 1.0) * (G.h / 2.0) : 0.0};
          double al = alpha_fe(P, xg);
          double jac = dim == 2 ? G.h / 2.0 : (G.h / 2.0) * (G.h / 2.0);
          double Na = shape_fn(dim, a, xi);
          if (Na == 0.0) continue;
          py += al * Na * ty * jac * thick;
        }
      }
    }
  }
  // uniform traction (+x) on the face x = dom_hi: elements of the last column, face xi = +1
  if (Tx != 0.0) {
    for (int t = n2e_ptr[n]; t < n2e_ptr[n + 1]; t++) {
      int64_t e = n2e[t] / nen;
      int a = n2e[t] % nen;
      if (!eact[e]) continue;
      int64_t ex = e % G.ne[0], ey = (e / G.ne[0]) % G.ne[1], ez = e / (G.ne[0] * G.ne[1]);
      if (ex != G.ne[0] - 1) continue;
      int ngp2 = dim == 2 ? 2 : 4;
      for (int g = 0; g < ngp2; g++) {
        double xi[3] = {1.0, (g & 1) ? q : -q, (g & 2) ? q : -q};
        double xg[3] = {dom_hi_x, G.lo[1] + (double)ey * G.h + (xi[1] + 1.0) * (G.h / 2.0),
                        dim == 3 ? G.lo[2] + (double)ez * G.h + (xi[2] + 1.0) * (G.h / 2.0) : 0.0};
        double al = alpha_fe(P, xg);
        double jac = dim == 2 ? G.h / 2.0 : (G.h / 2.0) * (G.h / 2.0);
        double Na = shape_fn(dim, a, xi);
        if (Na == 0.0) continue;
        px += al * Na * Tx * jac * thick;
      }
    }
  }
  mF[n] = m;
  nact[n] = (uint8_t)act;
  for (int d = 0; d < dim; d++) PF[n * dim + d] = (d == 1) ? py : (d == 0) ? px : 0.0;
}

__global__ void k_fe_init(int64_t nfe, int dim, const uint8_t *nact, const uint8_t *bc, const double *PF,
                          const double *mF, double vbc, double *vF, double *aF) {
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nfe || !nact[n]) return;
  for (int d = 0; d < dim; d++) {
    int64_t t = n * dim + d;
    if (bc[t]) {
      vF[t] = vbc;
      aF[t] = 0.0;
    } else {
      aF[t] = PF[t] / mF[n];
    }
  }
}

template <int DIM, bool PRED>
__global__ void k_fe_elem_force(FeElemArgs E) {
  fe_elem_force_one<DIM, PRED>(E, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void k_fe_gather_free(FeGatherArgs G) { fe_gather_free_one(G, (int64_t)blockIdx.x * blockDim.x + threadIdx.x); }

__global__ void k_fe_correct_ring(FeRingArgs R) {
  fe_correct_ring_wave(R, ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE, (int)(threadIdx.x & (WAVE - 1)));
}

inline unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

MeshGeo mesh_geo(const Solver &s) {
  MeshGeo G{};
  for (int a = 0; a < 3; a++) {
    G.lo[a] = a < s.dim ? s.p.dom_lo[a] : 0.0;
    G.ne[a] = a < s.dim ? s.p.fe_n[a] : 1;
  }
  G.h = s.p.fe_h;
  return G;
}

}  // namespace

// Mesh topology (integer bookkeeping) on the host; every floating-point
// quantity (weights, masses, loads, forces) on the device.
void fe_setup(Solver &s) {
  const int dim = s.dim;
  const mts_problem &p = s.p;
  hipStream_t st = s.stream;
  s.nen = dim == 2 ? 4 : 8;
  s.ngp = s.nen;
  s.nstr = dim == 2 ? 3 : 6;
  const int nen = s.nen;
  int64_t nx = p.fe_n[0], ny = p.fe_n[1], nz = dim == 3 ? p.fe_n[2] : 1;
  int64_t gx = nx + 1, gy = ny + 1, gz = dim == 3 ? nz + 1 : 1;
  int64_t ngrid = gx * gy * gz;
  s.ne = nx * ny * nz;
  double h = p.fe_h;
  // slit nodes on crack lines (2D): grid nodes with x_start <= x < x_end are duplicated;
  // elements whose lower edge lies on the line use the copy.
  std::vector<int64_t> dup(ngrid, -1);
  int64_t nfe = ngrid;
  for (int c = 0; c < p.n_cracks && dim == 2; c++) {
    double jf = (p.cracks[c][0] - p.dom_lo[1]) / h;
    int64_t jc = (int64_t)std::llround(jf);
    if (std::fabs(jf - (double)jc) > 1e-6 || jc <= 0 || jc >= ny)
      throw ArgError{"crack line is not an interior FE node line"};
    for (int64_t i = 0; i <= nx; i++) {
      double xn = p.dom_lo[0] + (double)i * h;
      if (xn >= p.cracks[c][1] - 1e-9 * h && xn < p.cracks[c][2] - 1e-9 * h) {
        int64_t g = jc * gx + i;
        if (dup[g] < 0) dup[g] = nfe++;
      }
    }
  }
  s.nfe = nfe;
  s.h_conn.assign((size_t)(s.ne * nen), 0);
  const int q4[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
  for (int64_t ez = 0; ez < nz; ez++)
    for (int64_t ey = 0; ey < ny; ey++)
      for (int64_t ex = 0; ex < nx; ex++) {
        int64_t e = (ez * ny + ey) * nx + ex;
        for (int a = 0; a < nen; a++) {
          int64_t i = ex + q4[a & 3][0], j = ey + q4[a & 3][1], k = ez + (a >= 4 ? 1 : 0);
          int64_t g = (k * gy + j) * gx + i;
          int64_t node = g;
          if (dup[g] >= 0 && q4[a & 3][1] == 0) node = dup[g];
          s.h_conn[e * nen + a] = (int32_t)node;
        }
      }
  // node -> (element*nen + local) in ascending element order
  std::vector<int32_t> cnt(nfe + 1, 0);
  for (int64_t e = 0; e < s.ne; e++)
    for (int a = 0; a < nen; a++) cnt[s.h_conn[e * nen + a] + 1]++;
  for (int64_t n = 0; n < nfe; n++) cnt[n + 1] += cnt[n];
  std::vector<int32_t> n2e(cnt[nfe]), fill(cnt.begin(), cnt.end() - 1);
  for (int64_t e = 0; e < s.ne; e++)
    for (int a = 0; a < nen; a++) n2e[fill[s.h_conn[e * nen + a]]++] = (int32_t)(e * nen + a);
  // prescribed x-velocity on the face x = dom_lo (grid column i = 0 and its slit copies)
  s.h_bc.assign((size_t)(nfe * dim), 0);
  if (p.clamp_x0) {  // fixed face x = dom_lo: every component (vel_bc = 0, so flagged dofs stay at rest)
    for (int64_t k = 0; k < gz; k++)
      for (int64_t j = 0; j < gy; j++) {
        int64_t g = (k * gy + j) * gx;
        for (int d = 0; d < dim; d++) {
          s.h_bc[g * dim + d] = 1;
          if (dup[g] >= 0) s.h_bc[dup[g] * dim + d] = 1;
        }
      }
  }
  if (p.vel_bc != 0.0) {
    for (int64_t k = 0; k < gz; k++)
      for (int64_t j = 0; j < gy; j++) {
        int64_t g = (k * gy + j) * gx;
        s.h_bc[g * dim] = 1;
        if (dup[g] >= 0) s.h_bc[dup[g] * dim] = 1;
      }
  }
  // device arrays
  DeviceArena &ar = s.arena;
  s.conn = ar.alloc<int32_t>(s.ne * nen);
  s.eact = ar.alloc<uint8_t>(s.ne);
  s.gpa = ar.alloc<double>(s.ne * s.ngp);
  s.n2e_ptr = ar.alloc<int32_t>(nfe + 1);
  s.n2e = ar.alloc<int32_t>(n2e.size());
  s.nact = ar.alloc<uint8_t>(nfe);
  s.bc = ar.alloc<uint8_t>(nfe * dim);
  s.mF = ar.alloc<double>(nfe);
  s.PF = ar.alloc<double>(nfe * dim);
  s.uF = ar.alloc<double>(nfe * dim);
  s.vF = ar.alloc<double>(nfe * dim);
  s.aF = ar.alloc<double>(nfe * dim);
  s.ut = ar.alloc<double>(nfe * dim);
  s.vt = ar.alloc<double>(nfe * dim);
  s.at = ar.alloc<double>(nfe * dim);
  s.fe_buf = ar.alloc<double>(s.ne * nen * dim);
  s.xF = ar.alloc<double>(nfe * dim);
  MTS_HIP(hipMemcpyAsync(s.conn, s.h_conn.data(), sizeof(int32_t) * s.ne * nen, hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemcpyAsync(s.n2e_ptr, cnt.data(), sizeof(int32_t) * (nfe + 1), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemcpyAsync(s.n2e, n2e.data(), sizeof(int32_t) * n2e.size(), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemcpyAsync(s.bc, s.h_bc.data(), nfe * dim, hipMemcpyHostToDevice, st));
  for (double *q : {s.uF, s.vF, s.aF, s.ut, s.vt, s.at})
    MTS_HIP(hipMemsetAsync(q, 0, sizeof(double) * nfe * dim, st));
  // node coordinates (grid positions; slit copies share them) -- host layout data
  std::vector<double> xf((size_t)(nfe * dim));
  for (int64_t k = 0; k < gz; k++)
    for (int64_t j = 0; j < gy; j++)
      for (int64_t i = 0; i < gx; i++) {
        int64_t g = (k * gy + j) * gx + i;
        double c[3] = {p.dom_lo[0] + (double)i * h, p.dom_lo[1] + (double)j * h, dim == 3 ? p.dom_lo[2] + (double)k * h : 0};
        for (int d = 0; d < dim; d++) {
          xf[g * dim + d] = c[d];
          if (dup[g] >= 0) xf[dup[g] * dim + d] = c[d];
        }
      }
  MTS_HIP(hipMemcpyAsync(s.xF, xf.data(), sizeof(double) * nfe * dim, hipMemcpyHostToDevice, st));

  FeTables *tab = ar.alloc<FeTables>(1);
  k_fe_tables<<<1, 1, 0, st>>>(dim, h, p.E, dim == 2 ? 1.0 / 3.0 : 0.25, tab);
  MTS_LAUNCH_CHECK();
  s.fe_tab = tab;  // per solver: solvers of different mesh sizes coexist
  MeshGeo G = mesh_geo(s);
  k_fe_gp_alpha<<<nb(s.ne), 256, 0, st>>>(s.prm, G, s.ne, s.ngp, s.gpa, s.eact);
  MTS_LAUNCH_CHECK();
  k_fe_node_setup<<<nb(nfe), 256, 0, st>>>(s.prm, G, nfe, nen, s.ngp, s.n2e_ptr, s.n2e, s.gpa, s.eact, p.traction,
                                           p.dom_hi[1], p.traction_x, p.dom_hi[0], p.thickness, s.mF, s.PF, s.nact,
                                           tab);
  MTS_LAUNCH_CHECK();
  k_fe_init<<<nb(nfe), 256, 0, st>>>(nfe, dim, s.nact, s.bc, s.PF, s.mF, p.vel_bc, s.vF, s.aF);
  MTS_LAUNCH_CHECK();
  MTS_HIP(hipStreamSynchronize(st));
  if (s.fe_beta > 0.0) fe_implicit_setup(s);
}

FeElemArgs fe_elem_args(Solver &s, bool predict) {
  FeElemArgs E{};
  E.ne = s.ne;
  E.conn = s.conn;
  E.eact = s.eact;
  E.gpa = s.gpa;
  E.u = s.uF;
  if (predict) {
    E.v = s.vF;
    E.acc = s.aF;
    E.bc = s.bc;
    E.dt = s.prm.dtF;
    E.hdt2 = s.prm.hdt2F;
    E.vbc = s.p.vel_bc;
  }
  E.thick = s.p.thickness;
  E.tab = static_cast<const FeTables *>(s.fe_tab);
  E.fe_buf = s.fe_buf;
  return E;
}

FeGatherArgs fe_gather_args(Solver &s) {
  FeGatherArgs G{};
  G.nfe = s.nfe;
  G.dim = s.dim;
  G.nen = s.nen;
  G.n2e_ptr = s.n2e_ptr;
  G.n2e = s.n2e;
  G.eact = s.eact;
  G.nact = s.nact;
  G.bc = s.bc;
  G.fe_buf = s.fe_buf;
  G.PF = s.PF;
  G.mF = s.mF;
  G.v = s.vF;
  G.a = s.aF;
  G.dt = s.prm.dtF;
  G.hdt2 = s.prm.hdt2F;
  G.hdt = s.prm.hdtF;
  G.vbc = s.p.vel_bc;
  G.at = s.at;
  G.vt = s.vt;
  G.f2c_ptr = s.f2c_ptr;
  G.ut = s.ut;
  G.u = s.uF;
  return G;
}

FeRingArgs fe_ring_args(Solver &s) {
  FeRingArgs R{};
  R.n_ring = s.n_ring;
  R.ring = s.fe_ring;
  R.dim = s.dim;
  R.nen = s.nen;
  R.bc = s.bc;
  R.f2c_ptr = s.f2c_ptr;
  R.f2c = s.f2c;
  R.cw = s.cw;
  R.lam = s.lam;
  R.mF = s.mF;
  R.ut = s.ut;
  R.vt = s.vt;
  R.at = s.at;
  R.hdt = s.prm.hdtF;
  R.uF = s.uF;
  R.vF = s.vF;
  R.aF = s.aF;
  return R;
}

void fe_free_step(Solver &s) {
  if (s.fe_beta > 0.0) return fe_implicit_free_step(s);
  hipStream_t st = s.stream;
  const FeElemArgs E = fe_elem_args(s, true);
  if (s.dim == 2) k_fe_elem_force<2, true><<<nb(s.ne), 256, 0, st>>>(E);
  else k_fe_elem_force<3, true><<<nb(s.ne), 256, 0, st>>>(E);
  MTS_LAUNCH_CHECK();
  k_fe_gather_free<<<nb(s.nfe), 256, 0, st>>>(fe_gather_args(s));
  MTS_LAUNCH_CHECK();
}

// Element forces of the current (corrected) FE displacement into fe_buf
// (inspection: energies).  fe_buf is free between macro steps.
void fe_elem_forces_current(Solver &s) {
  hipStream_t st = s.stream;
  const FeElemArgs E = fe_elem_args(s, false);
  if (s.dim == 2) k_fe_elem_force<2, false><<<nb(s.ne), 256, 0, st>>>(E);
  else k_fe_elem_force<3, false><<<nb(s.ne), 256, 0, st>>>(E);
  MTS_LAUNCH_CHECK();
}

void fe_correct(Solver &s) {
  if (s.fe_beta > 0.0) return fe_implicit_correct(s);
  if (!s.n_ring) return;
  k_fe_correct_ring<<<(unsigned)((s.n_ring * WAVE + 255) / 256), 256, 0, s.stream>>>(fe_ring_args(s));
  MTS_LAUNCH_CHECK();
}

}  // namespace mts
