// Implicit PD step (Newmark gamma = 1/2, beta = 1/4, Eq. 38 applied to the PD
// subdomain; pure-PD mode, FP64).
//
// Each step: u* = u + dt v + (1/2 - beta) dt^2 a, then (M + beta dt^2 K) a' =
// P + f(u*) with the linear bond force of Eq. 2 (K u = -f(u)) and the current
// bond states, u' = u* + beta dt^2 a', v' = v + dt/2 (a + a'), a = a'.  The
// critical-stretch test (Eq. 3-4) then runs on u' and its breaks take effect
// from the next step.  The operator is applied matrix-free over the
// full-lattice sliced layout (one wavefront per slice, L lanes per row, a fixed
// shuffle order, so sums are deterministic) and the system is solved by the
// Jacobi-preconditioned conjugate gradients of cg1.h.
#include "cg1.h"
#include "device_math.h"

#include <cmath>
#include <vector>

namespace mts {

namespace {

inline unsigned nbp(int64_t n) { return (unsigned)((n + 255) / 256); }

struct PdiArgs {
  const double *x;  // positions [dim][N]
  const int32_t *rows, *width, *col;
  const int64_t *slot_off, *word_off;
  const uint64_t *mask;
  const double *coef, *mass;
  int64_t N, n_rows, n_slices;
};

// Row sums of the linear bond force f_i(in) = sum_k coef (xi . (in_k - in_i)) xi
// over intact bonds, with in_k = in[k * stride + off + d]; lane l of the row
// adds slots l, l + L, ... and the row's lanes are combined by a fixed butterfly.
template <int DIM, int L>
__device__ inline void row_force(const PdiArgs &A, int64_t slice, int64_t i, bool valid, const double *in, int stride,
                                 int off, double F[DIM]) {
  const int lane = threadIdx.x & (WAVE - 1);
  for (int d = 0; d < DIM; d++) F[d] = 0.0;
  if (valid) {
    const int T = A.width[slice] / L;
    double ui[DIM], xi_[DIM];
    for (int d = 0; d < DIM; d++) {
      ui[d] = in[i * stride + off + d];
      xi_[d] = A.x[d * A.N + i];
    }
    for (int t = 0; t < T; t++) {
      if (!((A.mask[A.word_off[slice] + t] >> lane) & 1ull)) continue;
      const int64_t pos = A.slot_off[slice] + (int64_t)t * WAVE + lane;
      const int64_t c = A.col[pos];
      const double cf = A.coef[pos];
      double xi[DIM], xe = 0.0;
      for (int d = 0; d < DIM; d++) {
        xi[d] = A.x[d * A.N + c] - xi_[d];
        xe += xi[d] * (in[c * stride + off + d] - ui[d]);
      }
      for (int d = 0; d < DIM; d++) F[d] += (cf * xe) * xi[d];
    }
  }
  for (int o = L / 2; o >= 1; o >>= 1)
    for (int d = 0; d < DIM; d++) F[d] += __shfl_xor(F[d], o, WAVE);
}

// y_t = P_t + ms m_i in_t + ks (K in)_t with K in = -f(in), t = i dim + d; with
// part, also per-workgroup partial sums of in . y (the operator's p.q).
template <int DIM, int L>
__global__ __launch_bounds__(256) void k_pdi_apply(PdiArgs A, const int32_t *state, const double *in, int stride,
                                                   int off, const double *P, double ms, double ks, double *y,
                                                   double *part) {
  __shared__ double lds[256];
  if (state && state[0]) return;  // the solve has converged
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t slice = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int S = WAVE / L, jl = lane / L, l = lane % L;
  const int64_t r = slice * S + jl;
  const bool valid = slice < A.n_slices && r < A.n_rows;
  const int64_t i = valid ? A.rows[r] : 0;
  double F[DIM];
  row_force<DIM, L>(A, slice, i, valid, in, stride, off, F);
  double v = 0.0;
  if (valid && l == 0) {
    for (int d = 0; d < DIM; d++) {
      const double xin = in[i * stride + off + d];
      double yv = ms * (A.mass[i] * xin) - ks * F[d];
      if (P) yv = P[d * A.N + i] + yv;
      y[i * DIM + d] = yv;
      v += xin * yv;
    }
  }
  if (part) {
    const double sum = block_tree(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = sum;
  }
}

// Jacobi preconditioner: 1 / (m_i + c sum_k coef xi_d^2) over intact bonds.
template <int DIM, int L>
__global__ __launch_bounds__(256) void k_pdi_diag(PdiArgs A, double c, double *inv_diag) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t slice = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int S = WAVE / L, jl = lane / L, l = lane % L;
  const int64_t r = slice * S + jl;
  const bool valid = slice < A.n_slices && r < A.n_rows;
  const int64_t i = valid ? A.rows[r] : 0;
  double D[DIM];
  for (int d = 0; d < DIM; d++) D[d] = 0.0;
  if (valid) {
    const int T = A.width[slice] / L;
    for (int t = 0; t < T; t++) {
      if (!((A.mask[A.word_off[slice] + t] >> lane) & 1ull)) continue;
      const int64_t pos = A.slot_off[slice] + (int64_t)t * WAVE + lane;
      const int64_t k = A.col[pos];
      for (int d = 0; d < DIM; d++) {
        const double xd = A.x[d * A.N + k] - A.x[d * A.N + i];
        D[d] += A.coef[pos] * (xd * xd);
      }
    }
  }
  for (int o = L / 2; o >= 1; o >>= 1)
    for (int d = 0; d < DIM; d++) D[d] += __shfl_xor(D[d], o, WAVE);
  if (valid && l == 0)
    for (int d = 0; d < DIM; d++) inv_diag[i * DIM + d] = 1.0 / (A.mass[i] + c * D[d]);
}

// u* = (u + dt v) + b2 a into the u part of the other node records.
__global__ void k_pdi_predict(int64_t N, int dim, double dt, double b2, const double *xu, const double *v,
                              const double *a, double *xu_next) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  for (int d = 0; d < dim; d++) {
    const int64_t t = d * N + i, q = i * 2 * dim + dim + d;
    xu_next[q] = (xu[q] + dt * v[t]) + b2 * a[t];
  }
}

// u' = u* + c a', v' = v + dt/2 (a + a'), a = a'; a non-finite velocity sets
// the instability flag.
__global__ void k_pdi_post(int64_t N, int dim, double c, double hdt, const double *an, double *xu_next, double *v,
                           double *a, int32_t *nonfinite) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  bool bad = false;
  for (int d = 0; d < dim; d++) {
    const int64_t t = d * N + i, q = i * 2 * dim + dim + d;
    const double x = an[i * dim + d];
    xu_next[q] = xu_next[q] + c * x;
    const double vn = v[t] + hdt * (a[t] + x);
    v[t] = vn;
    a[t] = x;
    if (!std::isfinite(vn)) bad = true;
  }
  if (bad) nonfinite[0] = 1;
}

// Critical-stretch test (Eq. 3-4) on the displacement of the node records;
// the wavefront clears the bits of its bonds that break in its own mask words.
template <int DIM, int L>
__global__ __launch_bounds__(256) void k_pdi_break(PdiArgs A, const double *xu, double K2, double scrit,
                                                   uint64_t *mask) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t slice = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (slice >= A.n_slices) return;  // uniform per wavefront
  const int S = WAVE / L, jl = lane / L;
  const int64_t r = slice * S + jl;
  const bool valid = r < A.n_rows;
  const int64_t i = valid ? A.rows[r] : 0;
  const int T = A.width[slice] / L;
  for (int t = 0; t < T; t++) {
    const uint64_t word = A.mask[A.word_off[slice] + t];
    bool cut = false;
    if (valid && ((word >> lane) & 1ull)) {
      const int64_t pos = A.slot_off[slice] + (int64_t)t * WAVE + lane;
      const int64_t c = A.col[pos];
      double xi[DIM], eta[DIM];
      for (int d = 0; d < DIM; d++) {
        xi[d] = xu[c * 2 * DIM + d] - xu[i * 2 * DIM + d];
        eta[d] = xu[c * 2 * DIM + DIM + d] - xu[i * 2 * DIM + DIM + d];
      }
      // squared lengths as the plain formula forms them (no contraction)
      double r2 = xi[0] * xi[0] + xi[1] * xi[1];
      const double y0 = xi[0] + eta[0], y1 = xi[1] + eta[1];
      double y2 = y0 * y0 + y1 * y1;
      if (DIM == 3) {
        const double yz = xi[2] + eta[2];
        r2 = r2 + xi[2] * xi[2];
        y2 = y2 + yz * yz;
      }
      cut = breaks(r2, y2, K2, scrit);
    }
    const uint64_t cuts = __ballot(cut);
    if (cuts && lane == 0) mask[A.word_off[slice] + t] = word & ~cuts;
  }
}

}  // namespace

struct PdImplicit {
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *b = nullptr, *inv_diag = nullptr;
  double *part_pq = nullptr, *part_rz0 = nullptr, *part_rz[2] = {nullptr, nullptr};
  int32_t *state = nullptr, *h_state = nullptr;
  int64_t iters_last = 0;
};

namespace {

PdiArgs pdi_args(Solver &s) {
  PdiArgs A{};
  A.x = s.x;
  A.rows = s.sell.rows;
  A.width = s.sell.width;
  A.col = s.sell.col;
  A.slot_off = s.sell.slot_off;
  A.word_off = s.sell.word_off;
  A.mask = s.sell.mask;
  A.coef = s.sell.coef;
  A.mass = s.mass;
  A.N = s.N;
  A.n_rows = s.sell.n_rows;
  A.n_slices = s.sell.n_slices;
  return A;
}

#define MTS_PDI_BY(dim, L, MACRO)                                                          \
  if (dim == 2) {                                                                          \
    if (L == 1) MACRO(2, 1); else if (L == 2) MACRO(2, 2); else if (L == 4) MACRO(2, 4); else MACRO(2, 8); \
  } else {                                                                                 \
    if (L == 1) MACRO(3, 1); else if (L == 2) MACRO(3, 2); else if (L == 4) MACRO(3, 4); else MACRO(3, 8); \
  }

}  // namespace

void pd_implicit_setup(Solver &s) {
  if (!(s.pd_beta > 0.0)) return;
  if (!s.sell.coef || !s.sell.col) throw ArgError{"implicit PD: the bond layout keeps no coefficients"};
  PdImplicit *F = new PdImplicit();
  s.pd_impl = F;
  DeviceArena &ar = s.arena;
  const int64_t n = s.N * s.dim;
  for (double **b : {&F->x, &F->r, &F->z, &F->p, &F->q, &F->b, &F->inv_diag}) *b = ar.alloc<double>(n);
  const int64_t ga = (s.sell.n_slices + 3) / 4;
  F->part_pq = ar.alloc<double>(std::max<int64_t>(ga, 1));
  F->part_rz0 = ar.alloc<double>(nbp(n));
  F->part_rz[0] = ar.alloc<double>(nbp(n));
  F->part_rz[1] = ar.alloc<double>(nbp(n));
  F->state = ar.alloc<int32_t>(2);
  MTS_HIP(hipHostMalloc((void **)&F->h_state, 2 * sizeof(int32_t), hipHostMallocDefault));
}

void pd_implicit_step(Solver &s) {
  PdImplicit &F = *s.pd_impl;
  hipStream_t st = s.stream;
  const int dim = s.dim, L = s.sell.L;
  const int64_t N = s.N, n = N * dim;
  const double dt = s.prm.dtP, c = s.pd_beta * dt * dt, b2 = (0.5 - s.pd_beta) * dt * dt;
  const PdiArgs A = pdi_args(s);
  const unsigned ga = (unsigned)std::max<int64_t>((s.sell.n_slices + 3) / 4, 1);
  double *xn = s.xu[s.cur ^ 1];
  k_pdi_predict<<<nbp(N), 256, 0, st>>>(N, dim, dt, b2, s.xu[s.cur], s.v, s.a, xn);
  MTS_LAUNCH_CHECK();
  // b = P + f(u*) and the preconditioner (bond states as they are now)
#define MTS_RHS(D, LL) k_pdi_apply<D, LL><<<ga, 256, 0, st>>>(A, nullptr, xn, 2 * D, D, s.P, 0.0, -1.0, F.b, nullptr)
  MTS_PDI_BY(dim, L, MTS_RHS);
#undef MTS_RHS
  MTS_LAUNCH_CHECK();
#define MTS_DIAG(D, LL) k_pdi_diag<D, LL><<<ga, 256, 0, st>>>(A, c, F.inv_diag)
  MTS_PDI_BY(dim, L, MTS_DIAG);
#undef MTS_DIAG
  MTS_LAUNCH_CHECK();
  Cg1 C{};
  C.ndof = n;
  C.nblk = nbp(n);
  C.nblk_pq = ga;
  C.inv_diag = F.inv_diag;
  C.x = F.x;
  C.r = F.r;
  C.z = F.z;
  C.p = F.p;
  C.q = F.q;
  C.part_pq = F.part_pq;
  C.part_rz0 = F.part_rz0;
  C.part_rz[0] = F.part_rz[0];
  C.part_rz[1] = F.part_rz[1];
  C.state = F.state;
  C.tol = 1e-28;
  F.iters_last = cg1_run(st, C, F.b, F.iters_last, F.h_state, [&] {
#define MTS_OP(D, LL) k_pdi_apply<D, LL><<<ga, 256, 0, st>>>(A, F.state, F.p, D, 0, nullptr, 1.0, c, F.q, F.part_pq)
    MTS_PDI_BY(dim, L, MTS_OP);
#undef MTS_OP
    MTS_LAUNCH_CHECK();
  });
  k_pdi_post<<<nbp(N), 256, 0, st>>>(N, dim, c, s.prm.hdtP, F.x, xn, s.v, s.a, s.nonfinite_flag);
  MTS_LAUNCH_CHECK();
  s.cur ^= 1;
  if (s.breaking) {
#define MTS_BRK(D, LL) k_pdi_break<D, LL><<<ga, 256, 0, st>>>(A, s.xu[s.cur], s.prm.K2, s.prm.scrit, s.sell.mask)
    MTS_PDI_BY(dim, L, MTS_BRK);
#undef MTS_BRK
    MTS_LAUNCH_CHECK();
  }
  pd_damage(s);
  s.pd_steps++;
}

void pd_implicit_free(Solver &s) {
  if (!s.pd_impl) return;
  if (s.pd_impl->h_state) (void)hipHostFree(s.pd_impl->h_state);
  delete s.pd_impl;
  s.pd_impl = nullptr;
}

}  // namespace mts
