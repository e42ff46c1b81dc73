// Implicit FE step (Newmark gamma = 1/2, beta = 1/4, Eq. 38) at dt_FE = m dt_PD.
//
// With beta > 0 each FE step solves A a = b with A = M + beta dt^2 K (lumped
// weighted M, Arlequin-weighted K of Eq. 34) on the free dofs and the identity
// on prescribed and inactive dofs (their acceleration is zero):
//  - free problem (Eq. 47a): u* = u + dt v + (1/2 - beta) dt^2 a, A a~ = P - K u*,
//    u~ = u* + beta dt^2 a~, v~ = v + dt/2 a + dt/2 a~;
//  - link problem (Eq. 47b): A da = -G_F^T lambda, so the final update (Eq. 50)
//    adds (beta dt^2 da, dt/2 da, da), and the FE block of the multiplier
//    matrix (Eq. 49) is (dt/2) G_F A^-1 G_F^T.
// A is applied matrix-free from per-element stiffness matrices, gathered per
// dof in a fixed order, and solved by Jacobi-preconditioned conjugate
// gradients with fixed-order dot products (deterministic), several right-hand
// sides at once (vectors [dof][R]).
#include "fe_device.h"
#include "cg1.h"

#include <cmath>
#include <vector>

namespace mts {

namespace {

constexpr int kT = 256;

inline unsigned nbk(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

// K_e = sum_gp alpha B^T D B detJ t of every active element, row-major over
// (local node, component) pairs.
template <int DIM>
__global__ void k_fe_elem_matrix(int64_t ne, const uint8_t *eact, const double *gpa, const FeTables *tab, double thick,
                                 double *Ke) {
  constexpr int NEN = DIM == 2 ? 4 : 8, NSTR = DIM == 2 ? 3 : 6, ND = NEN * DIM;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double *K = Ke + e * ND * ND;
  for (int t = 0; t < ND * ND; t++) K[t] = 0.0;
  if (!eact[e]) return;
  for (int g = 0; g < NEN; g++) {
    const double al = gpa[e * NEN + g];
    if (al == 0.0) continue;
    const double scale = al * tab->detJ * thick;
    // B (NSTR x ND) at this Gauss point
    double B[NSTR][ND];
    for (int r = 0; r < NSTR; r++)
      for (int c = 0; c < ND; c++) B[r][c] = 0.0;
    for (int a = 0; a < NEN; a++) {
      const double *dN = tab->dN[g][a];
      if (DIM == 2) {
        B[0][a * 2] = dN[0];
        B[1][a * 2 + 1] = dN[1];
        B[2][a * 2] = dN[1];
        B[2][a * 2 + 1] = dN[0];
      } else {
        B[0][a * 3] = dN[0];
        B[1][a * 3 + 1] = dN[1];
        B[2][a * 3 + 2] = dN[2];
        B[3][a * 3] = dN[1];
        B[3][a * 3 + 1] = dN[0];
        B[4][a * 3 + 1] = dN[2];
        B[4][a * 3 + 2] = dN[1];
        B[5][a * 3] = dN[2];
        B[5][a * 3 + 2] = dN[0];
      }
    }
    for (int c = 0; c < ND; c++) {
      double DB[NSTR];
      for (int r = 0; r < NSTR; r++) {
        double t = 0.0;
        for (int k = 0; k < NSTR; k++) t += tab->D[r][k] * B[k][c];
        DB[r] = t;
      }
      for (int r = 0; r < ND; r++) {
        double t = 0.0;
        for (int k = 0; k < NSTR; k++) t += B[k][r] * DB[k];
        K[r * ND + c] += scale * t;
      }
    }
  }
}

struct ApplyArgs {
  int64_t ndof;
  int R, dim, nen;
  const double *Ke;
  const int32_t *n2e_ptr, *n2e, *conn;
  const uint8_t *eact, *freedof;
  const double *mF;
  const double *x;  // [ndof][R]
  double *y;        // [ndof][R]
  double ms, ks;    // y = P + ms M x + ks K x on free dofs
  const double *P;  // [ndof] or nullptr
};

// One (dof, RHS) per thread: the row of K gathered over the node's elements
// in ascending element order.  Free dofs: y = P + ms M x + ks K x; other dofs:
// y = x when ms != 0 (identity rows of A), else 0.
__global__ void k_fe_apply(ApplyArgs A) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= A.ndof * A.R) return;
  const int64_t t = id / A.R;
  const int r = (int)(id % A.R);
  if (!A.freedof[t]) {
    A.y[id] = A.ms != 0.0 ? A.x[id] : 0.0;
    return;
  }
  const int dim = A.dim, nen = A.nen, nd = nen * dim;
  const int64_t n = t / dim;
  const int dd = (int)(t % dim);
  double acc = 0.0;
  for (int k = A.n2e_ptr[n]; k < A.n2e_ptr[n + 1]; k++) {
    const int64_t e = A.n2e[k] / nen;
    const int la = A.n2e[k] % nen;
    if (!A.eact[e]) continue;
    const double *Krow = A.Ke + e * nd * nd + (int64_t)(la * dim + dd) * nd;
    for (int b = 0; b < nen; b++) {
      const int64_t nb = A.conn[e * nen + b];
      for (int db = 0; db < dim; db++) acc += Krow[b * dim + db] * A.x[(nb * dim + db) * A.R + r];
    }
  }
  double v = A.ks * acc;
  if (A.ms != 0.0) v = A.ms * A.mF[n] * A.x[id] + v;
  if (A.P) v = A.P[t] + v;
  A.y[id] = v;
}

// Diagonal of A (Jacobi preconditioner): M + c K_tt on free dofs, 1 elsewhere.
__global__ void k_fe_diag(int64_t ndof, int dim, int nen, const double *Ke, const int32_t *n2e_ptr, const int32_t *n2e,
                          const uint8_t *eact, const uint8_t *freedof, const double *mF, double c, double *inv_diag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ndof) return;
  if (!freedof[t]) {
    inv_diag[t] = 1.0;
    return;
  }
  const int nd = nen * dim;
  const int64_t n = t / dim;
  const int dd = (int)(t % dim);
  double k = 0.0;
  for (int q = n2e_ptr[n]; q < n2e_ptr[n + 1]; q++) {
    const int64_t e = n2e[q] / nen;
    const int la = n2e[q] % nen;
    if (!eact[e]) continue;
    k += Ke[e * nd * nd + (int64_t)(la * dim + dd) * nd + la * dim + dd];
  }
  inv_diag[t] = 1.0 / (mF[n] + c * k);
}

__global__ void k_fe_freedof(int64_t nfe, int dim, const uint8_t *nact, const uint8_t *bc, uint8_t *freedof) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nfe * dim) freedof[t] = (nact[t / dim] && !bc[t]) ? 1 : 0;
}

// Per-workgroup partial sums of a_i b_i for every RHS: part[blk * R + r].
__global__ __launch_bounds__(kT) void k_dot_part(int64_t ndof, int R, const double *a, const double *b, double *part) {
  __shared__ double lds[kT];
  for (int r = 0; r < R; r++) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = t < ndof ? a[t * R + r] * b[t * R + r] : 0.0;
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int h = kT / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) lds[threadIdx.x] += lds[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x * R + r] = lds[0];
    __syncthreads();
  }
}

// out[r] = sum over blocks of part[blk * R + r] in a fixed order (one
// workgroup per RHS).
__global__ __launch_bounds__(kT) void k_dot_final(const double *part, int64_t nblk, int R, double *out) {
  __shared__ double lds[kT];
  const int r = blockIdx.x;
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < nblk; k += kT) s += part[k * R + r];
  lds[threadIdx.x] = s;
  __syncthreads();
  for (int h = kT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) lds[threadIdx.x] += lds[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = lds[0];
}

// x += alpha p, r -= alpha q, z = D^-1 r with alpha = rz / pq (per RHS; 0 once
// that RHS has converged to an exact zero).
__global__ void k_cg_update(int64_t ndof, int R, const double *rz, const double *pq, const double *inv_diag,
                            const double *p, const double *q, double *x, double *r, double *z) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ndof * R) return;
  const int k = (int)(id % R);
  const double al = pq[k] > 0.0 ? rz[k] / pq[k] : 0.0;
  x[id] = x[id] + al * p[id];
  const double rn = r[id] - al * q[id];
  r[id] = rn;
  z[id] = rn * inv_diag[id / R];
}

// p = z + beta p with beta = rz_new / rz_old (per RHS).
__global__ void k_cg_dir(int64_t ndof, int R, const double *rz_new, const double *rz_old, const double *z, double *p) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ndof * R) return;
  const int k = (int)(id % R);
  const double be = rz_old[k] > 0.0 ? rz_new[k] / rz_old[k] : 0.0;
  p[id] = z[id] + be * p[id];
}

// start: x = 0, r = b, z = p = D^-1 b
__global__ void k_cg_init(int64_t ndof, int R, const double *b, const double *inv_diag, double *x, double *r, double *z,
                          double *p) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ndof * R) return;
  const double zi = b[id] * inv_diag[id / R];
  x[id] = 0.0;
  r[id] = b[id];
  z[id] = zi;
  p[id] = zi;
}

// Free problem predictor u* (free dofs), prescribed-velocity dofs move at vbc.
__global__ void k_fe_impl_pred(int64_t ndof, const uint8_t *freedof, const uint8_t *bc, const double *u, const double *v,
                               const double *a, double dt, double b2, double vbc, double *us) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ndof) return;
  if (freedof[t]) us[t] = (u[t] + dt * v[t]) + b2 * a[t];
  else us[t] = bc[t] ? u[t] + dt * vbc : u[t];
}

// u~ = u* + beta dt^2 a~, v~ = v + dt/2 a + dt/2 a~ on free dofs; prescribed
// dofs keep u*, v = vbc, a = 0.
__global__ void k_fe_impl_post(int64_t ndof, const uint8_t *freedof, const uint8_t *bc, const double *v,
                               const double *a, const double *sol, double c, double hdt, double vbc, double *ut,
                               double *vt, double *at) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ndof) return;
  if (freedof[t]) {
    const double an = sol[t];
    ut[t] = ut[t] + c * an;
    vt[t] = (v[t] + hdt * a[t]) + hdt * an;
    at[t] = an;
  } else {
    vt[t] = bc[t] ? vbc : v[t];
    at[t] = 0.0;
  }
}

// G_F^T lambda on the free dofs (fixed order over the node's constraint entries).
__global__ void k_fe_gft(int64_t ndof, int dim, int nen, const uint8_t *freedof, const int32_t *f2c_ptr,
                         const int32_t *f2c, const double *cw, const double *lam, double *out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ndof) return;
  double g = 0.0;
  if (freedof[t]) {
    const int64_t n = t / dim;
    const int d = (int)(t % dim);
    for (int k = f2c_ptr[n]; k < f2c_ptr[n + 1]; k++) {
      const int64_t q = f2c[k] / nen;
      const int aa = f2c[k] % nen;
      g += cw[q * nen + aa] * lam[q * dim + d];
    }
  }
  out[t] = g;
}

// Final FE update with the link response da = -A^-1 G_F^T lambda (sol holds
// A^-1 G_F^T lambda).
__global__ void k_fe_impl_corr(int64_t ndof, const double *sol, double c, double hdt, const double *ut, const double *vt,
                               const double *at, double *u, double *v, double *a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ndof) return;
  const double x = sol[t];
  u[t] = ut[t] - c * x;
  v[t] = vt[t] - hdt * x;
  a[t] = at[t] - x;
}

// Columns c0 .. c0 + R - 1 of G_F^T (free dofs), [ndof][R].
__global__ void k_fe_gft_cols(int64_t ndof, int R, int64_t c0, int64_t nl, int dim, int nen, const uint8_t *freedof,
                              const int32_t *f2c_ptr, const int32_t *f2c, const double *cw, double *out) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ndof * R) return;
  const int64_t t = id / R;
  const int64_t col = c0 + id % R;
  double g = 0.0;
  if (col < nl && freedof[t] && (int)(t % dim) == (int)(col % dim)) {
    const int64_t n = t / dim, qc = col / dim;
    for (int k = f2c_ptr[n]; k < f2c_ptr[n + 1]; k++)
      if (f2c[k] / nen == qc) g += cw[(int64_t)f2c[k]];
  }
  out[id] = g;
}

// HF[row, c0 + r] = dt/2 (G_F X)[row, r] for the solved columns X.
__global__ void k_hf_extract(int64_t nc, int dim, int nen, int64_t nl, int R, int64_t c0, const int32_t *cel,
                             const int32_t *conn, const double *cw, const double *X, double hdt, double *HF) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nc * dim * R) return;
  const int r = (int)(id % R);
  const int64_t row = id / R;
  if (c0 + r >= nl) return;
  const int64_t q = row / dim;
  const int d = (int)(row % dim);
  double g = 0.0;
  for (int a = 0; a < nen; a++) g += cw[q * nen + a] * X[((int64_t)conn[(int64_t)cel[q] * nen + a] * dim + d) * R + r];
  HF[row * nl + c0 + r] = hdt * g;
}

}  // namespace

// Buffers of the implicit step (allocated on first use by fe_implicit_setup).
// q = A p and partial sums of p.q
__global__ __launch_bounds__(kT) void k_cg1_apply(Cg1 C, ApplyArgs A) {
  __shared__ double lds[kT];
  if (C.state[0]) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (t < C.ndof) {
    double y;
    if (!A.freedof[t]) {
      y = C.p[t];
    } else {
      const int dim = A.dim, nen = A.nen, nd = nen * dim;
      const int64_t n = t / dim;
      const int dd = (int)(t % dim);
      double acc = 0.0;
      for (int k = A.n2e_ptr[n]; k < A.n2e_ptr[n + 1]; k++) {
        const int64_t e = A.n2e[k] / nen;
        const int la = A.n2e[k] % nen;
        if (!A.eact[e]) continue;
        const double *Krow = A.Ke + e * nd * nd + (int64_t)(la * dim + dd) * nd;
        for (int bb = 0; bb < nen; bb++) {
          const int64_t nb = A.conn[e * nen + bb];
          for (int db = 0; db < dim; db++) acc += Krow[bb * dim + db] * C.p[nb * dim + db];
        }
      }
      y = A.mF[n] * C.p[t] + A.ks * acc;
    }
    C.q[t] = y;
    v = C.p[t] * y;
  }
  const double sum = block_tree(v, lds);
  if (threadIdx.x == 0) C.part_pq[blockIdx.x] = sum;
}

struct FeImplicit {
  int R = 0;  // RHS capacity of the CG buffers
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *b = nullptr;
  double *part = nullptr, *rz0 = nullptr, *rz[2] = {nullptr, nullptr}, *pq = nullptr;
  double *us = nullptr;
  std::vector<double> h_rz0, h_rz;
  int64_t iters_last = 0;
  // one-RHS solver (the per-step solves)
  double *part_pq1 = nullptr, *part_rz0 = nullptr, *part_rz1[2] = {nullptr, nullptr};
  int32_t *state = nullptr, *h_state = nullptr;  // device flag and iteration count; pinned host copy
  int64_t iters1_last = 0;
};

void fe_implicit_setup(Solver &s) {
  const int64_t ndof = s.nfe * s.dim;
  const int nd = s.nen * s.dim;
  DeviceArena &ar = s.arena;
  hipStream_t st = s.stream;
  s.fe_Ke = ar.alloc<double>((size_t)s.ne * nd * nd);
  if (s.dim == 2) k_fe_elem_matrix<2><<<nbk(s.ne), kT, 0, st>>>(s.ne, s.eact, s.gpa, static_cast<const FeTables *>(s.fe_tab), s.p.thickness, s.fe_Ke);
  else k_fe_elem_matrix<3><<<nbk(s.ne), kT, 0, st>>>(s.ne, s.eact, s.gpa, static_cast<const FeTables *>(s.fe_tab), 1.0, s.fe_Ke);
  MTS_LAUNCH_CHECK();
  s.fe_free = ar.alloc<uint8_t>(ndof);
  k_fe_freedof<<<nbk(ndof), kT, 0, st>>>(s.nfe, s.dim, s.nact, s.bc, s.fe_free);
  MTS_LAUNCH_CHECK();
  s.fe_inv_diag = ar.alloc<double>(ndof);
  const double c = s.fe_beta * s.prm.dtF * s.prm.dtF;
  k_fe_diag<<<nbk(ndof), kT, 0, st>>>(ndof, s.dim, s.nen, s.fe_Ke, s.n2e_ptr, s.n2e, s.eact, s.fe_free, s.mF, c,
                                     s.fe_inv_diag);
  MTS_LAUNCH_CHECK();
  MTS_HIP(hipStreamSynchronize(st));
}

namespace {

FeImplicit &cg_buffers(Solver &s, int R) {
  if (!s.fe_impl) s.fe_impl = new FeImplicit();
  FeImplicit &F = *s.fe_impl;
  if (F.R >= R) return F;
  const int64_t ndof = s.nfe * s.dim;
  DeviceArena &ar = s.arena;
  for (double *q : {F.x, F.r, F.z, F.p, F.q, F.b, F.part, F.rz0, F.rz[0], F.rz[1], F.pq})
    if (q) ar.release(q);
  const size_t n = (size_t)ndof * R;
  F.x = ar.alloc<double>(n);
  F.r = ar.alloc<double>(n);
  F.z = ar.alloc<double>(n);
  F.p = ar.alloc<double>(n);
  F.q = ar.alloc<double>(n);
  F.b = ar.alloc<double>(n);
  F.part = ar.alloc<double>((size_t)nbk(ndof) * R);
  F.rz0 = ar.alloc<double>(R);
  F.rz[0] = ar.alloc<double>(R);
  F.rz[1] = ar.alloc<double>(R);
  F.pq = ar.alloc<double>(R);
  if (!F.us) F.us = ar.alloc<double>(ndof);
  if (!F.state) {
    const size_t nb = (size_t)nbk(ndof);
    F.part_pq1 = ar.alloc<double>(nb);
    F.part_rz0 = ar.alloc<double>(nb);
    F.part_rz1[0] = ar.alloc<double>(nb);
    F.part_rz1[1] = ar.alloc<double>(nb);
    F.state = ar.alloc<int32_t>(2);
    MTS_HIP(hipHostMalloc((void **)&F.h_state, 2 * sizeof(int32_t), hipHostMallocDefault));
  }
  F.R = R;
  return F;
}

void dot(Solver &s, FeImplicit &F, int R, const double *a, const double *b, double *out) {
  const int64_t ndof = s.nfe * s.dim;
  k_dot_part<<<nbk(ndof), kT, 0, s.stream>>>(ndof, R, a, b, F.part);
  MTS_LAUNCH_CHECK();
  k_dot_final<<<(unsigned)R, kT, 0, s.stream>>>(F.part, nbk(ndof), R, out);
  MTS_LAUNCH_CHECK();
}

ApplyArgs apply_args(Solver &s, int R, const double *x, double *y, double ms, double ks, const double *P) {
  ApplyArgs A{};
  A.ndof = s.nfe * s.dim;
  A.R = R;
  A.dim = s.dim;
  A.nen = s.nen;
  A.Ke = s.fe_Ke;
  A.n2e_ptr = s.n2e_ptr;
  A.n2e = s.n2e;
  A.conn = s.conn;
  A.eact = s.eact;
  A.freedof = s.fe_free;
  A.mF = s.mF;
  A.x = x;
  A.y = y;
  A.ms = ms;
  A.ks = ks;
  A.P = P;
  return A;
}

// Solve A X = F.b for R right-hand sides into F.x: preconditioned CG until
// every RHS's r.z fell below 1e-28 of its start (relative residual ~1e-14),
// checked on the host every 8 iterations.
void cg_solve(Solver &s, FeImplicit &F, int R) {
  const int64_t ndof = s.nfe * s.dim;
  hipStream_t st = s.stream;
  const double c = s.fe_beta * s.prm.dtF * s.prm.dtF;
  const unsigned g = nbk(ndof * R);
  k_cg_init<<<g, kT, 0, st>>>(ndof, R, F.b, s.fe_inv_diag, F.x, F.r, F.z, F.p);
  MTS_LAUNCH_CHECK();
  dot(s, F, R, F.r, F.z, F.rz0);
  MTS_HIP(hipMemcpyAsync(F.rz[0], F.rz0, sizeof(double) * R, hipMemcpyDeviceToDevice, st));
  F.h_rz0.resize(R);
  F.h_rz.resize(R);
  MTS_HIP(hipMemcpyAsync(F.h_rz0.data(), F.rz0, sizeof(double) * R, hipMemcpyDeviceToHost, st));
  MTS_HIP(hipStreamSynchronize(st));
  int cur = 0;
  int64_t it = 0;
  const int64_t max_it = 4000;
  for (;;) {
    for (int k = 0; k < 8; k++, it++) {
      k_fe_apply<<<g, kT, 0, st>>>(apply_args(s, R, F.p, F.q, 1.0, c, nullptr));
      MTS_LAUNCH_CHECK();
      dot(s, F, R, F.p, F.q, F.pq);
      k_cg_update<<<g, kT, 0, st>>>(ndof, R, F.rz[cur], F.pq, s.fe_inv_diag, F.p, F.q, F.x, F.r, F.z);
      MTS_LAUNCH_CHECK();
      dot(s, F, R, F.r, F.z, F.rz[cur ^ 1]);
      k_cg_dir<<<g, kT, 0, st>>>(ndof, R, F.rz[cur ^ 1], F.rz[cur], F.z, F.p);
      MTS_LAUNCH_CHECK();
      cur ^= 1;
    }
    MTS_HIP(hipMemcpyAsync(F.h_rz.data(), F.rz[cur], sizeof(double) * R, hipMemcpyDeviceToHost, st));
    MTS_HIP(hipStreamSynchronize(st));
    bool done = true;
    for (int k = 0; k < R; k++)
      if (!(F.h_rz[k] <= 1e-28 * F.h_rz0[k])) done = false;
    if (done) break;
    if (it >= max_it) throw ArgError{"implicit FE: conjugate gradients did not converge"};
  }
  F.iters_last = it;
}

// One right-hand side (x <- A^-1 b): three launches per iteration, the
// convergence flag read by the host after as many iterations as the previous
// solve needed plus one (at least kCgMinIters), then every eight.
void cg_solve1(Solver &s, FeImplicit &F) {
  const int64_t ndof = s.nfe * s.dim;
  hipStream_t st = s.stream;
  const unsigned g = nbk(ndof);
  Cg1 C{};
  C.ndof = ndof;
  C.nblk = g;
  C.nblk_pq = g;
  C.inv_diag = s.fe_inv_diag;
  C.x = F.x;
  C.r = F.r;
  C.z = F.z;
  C.p = F.p;
  C.q = F.q;
  C.part_pq = F.part_pq1;
  C.part_rz0 = F.part_rz0;
  C.part_rz[0] = F.part_rz1[0];
  C.part_rz[1] = F.part_rz1[1];
  C.state = F.state;
  C.tol = 1e-28;
  const ApplyArgs A = apply_args(s, 1, F.p, F.q, 1.0, s.fe_beta * s.prm.dtF * s.prm.dtF, nullptr);
  F.iters1_last = cg1_run(st, C, F.b, F.iters1_last, F.h_state, [&] {
    k_cg1_apply<<<g, kT, 0, st>>>(C, A);
    MTS_LAUNCH_CHECK();
  });
}

}  // namespace

void fe_implicit_free_step(Solver &s) {
  const int64_t ndof = s.nfe * s.dim;
  hipStream_t st = s.stream;
  FeImplicit &F = cg_buffers(s, 1);
  const double dt = s.prm.dtF, b2 = (0.5 - s.fe_beta) * dt * dt, c = s.fe_beta * dt * dt;
  k_fe_impl_pred<<<nbk(ndof), kT, 0, st>>>(ndof, s.fe_free, s.bc, s.uF, s.vF, s.aF, dt, b2, s.p.vel_bc, s.ut);
  MTS_LAUNCH_CHECK();
  k_fe_apply<<<nbk(ndof), kT, 0, st>>>(apply_args(s, 1, s.ut, F.b, 0.0, -1.0, s.PF));  // b = P - K u*
  MTS_LAUNCH_CHECK();
  cg_solve1(s, F);
  k_fe_impl_post<<<nbk(ndof), kT, 0, st>>>(ndof, s.fe_free, s.bc, s.vF, s.aF, F.x, c, s.prm.hdtF, s.p.vel_bc, s.ut,
                                            s.vt, s.at);
  MTS_LAUNCH_CHECK();
}

void fe_implicit_correct(Solver &s) {
  const int64_t ndof = s.nfe * s.dim;
  hipStream_t st = s.stream;
  FeImplicit &F = cg_buffers(s, 1);
  k_fe_gft<<<nbk(ndof), kT, 0, st>>>(ndof, s.dim, s.nen, s.fe_free, s.f2c_ptr, s.f2c, s.cw, s.lam0, F.b);
  MTS_LAUNCH_CHECK();
  cg_solve1(s, F);
  const double c = s.fe_beta * s.prm.dtF * s.prm.dtF;
  k_fe_impl_corr<<<nbk(ndof), kT, 0, st>>>(ndof, F.x, c, s.prm.hdtF, s.ut, s.vt, s.at, s.uF, s.vF, s.aF);
  MTS_LAUNCH_CHECK();
}

void fe_implicit_hf(Solver &s) {
  const int64_t ndof = s.nfe * s.dim, nl = s.nl;
  hipStream_t st = s.stream;
  const int R = (int)std::min<int64_t>(32, nl);
  FeImplicit &F = cg_buffers(s, R);
  if (!s.fe_HF) s.fe_HF = s.arena.alloc<double>((size_t)nl * nl);
  for (int64_t c0 = 0; c0 < nl; c0 += R) {
    k_fe_gft_cols<<<nbk(ndof * R), kT, 0, st>>>(ndof, R, c0, nl, s.dim, s.nen, s.fe_free, s.f2c_ptr, s.f2c, s.cw, F.b);
    MTS_LAUNCH_CHECK();
    cg_solve(s, F, R);
    k_hf_extract<<<nbk(s.nc * s.dim * R), kT, 0, st>>>(s.nc, s.dim, s.nen, nl, R, c0, s.cel, s.conn, s.cw, F.x,
                                                       s.prm.hdtF, s.fe_HF);
    MTS_LAUNCH_CHECK();
  }
  MTS_HIP(hipStreamSynchronize(st));
}

void fe_implicit_free(Solver &s) {
  if (s.fe_impl && s.fe_impl->h_state) (void)hipHostFree(s.fe_impl->h_state);
  delete s.fe_impl;
  s.fe_impl = nullptr;
}

}  // namespace mts
