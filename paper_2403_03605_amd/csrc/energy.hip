// Energies of the current state (inspection, not on the hot path):
//  - kinetic energy of the weighted masses, PD and FE (Eq. 17-18);
//  - PD deformation energy 1/4 sum_i sum_k mu w c (xi . eta)^2 V_i V_k (Eq. 6-7,
//    with the Arlequin bond weight w_ik);
//  - FE strain energy 1/2 u^T K_alpha u (Eq. 34), from the element forces;
//  - work of the constant loads P . u;
//  - bonds broken since setup (pre-crack cuts excluded).
// Each term is formed per node (or element) and summed in a fixed order.
#include <algorithm>
#include <cstring>

#include "device_math.h"

namespace mts {

void fe_elem_forces_current(Solver &s);

namespace {

constexpr int kRed = 256;

// terms[0][i] kinetic, [1][i] PD deformation, [2][i] load work of PD node i
__global__ void k_pd_energy_terms(int64_t N, int dim, const double *x, const double *xu, const double *v,
                                  const double *mass, const double *Pf, const int32_t *rp, const int32_t *row_of,
                                  int L, const int64_t *slot_off, const int32_t *col, const double *coef,
                                  const int64_t *word_off, const uint64_t *mask, double *terms) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double ui[3] = {0, 0, 0}, xi_[3] = {0, 0, 0}, ek = 0.0, w = 0.0;
  for (int d = 0; d < dim; d++) {
    ui[d] = xu[i * 2 * dim + dim + d];
    xi_[d] = x[d * N + i];
    const double vd = v[d * N + i];
    ek += 0.5 * mass[i] * vd * vd;
    if (Pf) w += Pf[d * N + i] * ui[d];
  }
  const int64_t r = row_of ? row_of[i] : i;
  const int S = WAVE / L;
  const int64_t sl = r / S;
  const int j = (int)(r % S);
  double e = 0.0;
  for (int k = 0; k < rp[i + 1] - rp[i]; k++) {
    if (!full_bit(word_off, mask, L, r, k)) continue;
    const int64_t pos = sell_slot(slot_off[sl], j, k, L);
    const int64_t c = col[pos];
    double xe = 0.0;
    for (int d = 0; d < dim; d++) xe += (x[d * N + c] - xi_[d]) * (xu[c * 2 * dim + dim + d] - ui[d]);
    e += coef[pos] * xe * xe;
  }
  terms[i] = ek;
  terms[N + i] = 0.25 * e;
  terms[2 * N + i] = w;
}

// terms[0][n] kinetic, [1][n] load work of FE node n (active nodes only)
__global__ void k_fe_node_terms(int64_t nfe, int dim, const uint8_t *nact, const double *u, const double *v,
                                const double *m, const double *PF, double *terms) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nfe) return;
  double ek = 0.0, w = 0.0;
  if (nact[n])
    for (int d = 0; d < dim; d++) {
      const double vd = v[n * dim + d];
      ek += 0.5 * m[n] * vd * vd;
      w += PF[n * dim + d] * u[n * dim + d];
    }
  terms[n] = ek;
  terms[nfe + n] = w;
}

// 1/2 u_e . f_e of every active element
__global__ void k_fe_elem_terms(int64_t ne, int nen, int dim, const int32_t *conn, const uint8_t *eact,
                                const double *u, const double *fe_buf, double *terms) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double s = 0.0;
  if (eact[e])
    for (int a = 0; a < nen; a++)
      for (int d = 0; d < dim; d++) s += u[(int64_t)conn[e * nen + a] * dim + d] * fe_buf[(e * nen + a) * dim + d];
  terms[e] = 0.5 * s;
}

// intact bonds: population count of the state words (padding bits are 0)
__global__ void k_popcount(const uint64_t *w, int64_t n, double *terms) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) terms[i] = (double)__popcll(w[i]);
}

// out[q] = sum of the n values of row q of terms, in a fixed order: thread t
// adds t, t + 256, ...; then a fixed tree.
__global__ __launch_bounds__(kRed) void k_sum_rows(const double *terms, int64_t n, double *out) {
  __shared__ double part[kRed];
  const int t = threadIdx.x;
  const double *row = terms + blockIdx.x * n;
  double s = 0.0;
  for (int64_t i = t; i < n; i += kRed) s += row[i];
  part[t] = s;
  __syncthreads();
  for (int h = kRed / 2; h > 0; h >>= 1) {
    if (t < h) part[t] += part[t + h];
    __syncthreads();
  }
  if (t == 0) out[blockIdx.x] = part[0];
}

inline unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

// sums of the rows (n values each) of a device terms array, to the host
void sum_rows(Solver &s, const double *terms, int rows, int64_t n, double *host_out) {
  double *dout = s.arena.alloc<double>(rows);
  k_sum_rows<<<(unsigned)rows, kRed, 0, s.stream>>>(terms, n, dout);
  MTS_LAUNCH_CHECK();
  MTS_HIP(hipMemcpyAsync(host_out, dout, sizeof(double) * rows, hipMemcpyDeviceToHost, s.stream));
  MTS_HIP(hipStreamSynchronize(s.stream));
  s.arena.release(dout);
}

}  // namespace

int64_t count_intact(Solver &s) {
  const int64_t n = std::max<int64_t>(s.sell.n_words, 1);
  double *t = s.arena.alloc<double>(n);
  k_popcount<<<nb(s.sell.n_words), 256, 0, s.stream>>>(s.sell.mask, s.sell.n_words, t);
  MTS_LAUNCH_CHECK();
  double c = 0.0;
  sum_rows(s, t, 1, s.sell.n_words, &c);
  s.arena.release(t);
  return (int64_t)c;
}

void energy_impl(Solver &s, mts_energy_info *o) {
  std::memset(o, 0, sizeof *o);
  const int64_t N = s.N;
  {
    double *t = s.arena.alloc<double>((size_t)3 * N);
    k_pd_energy_terms<<<nb(N), 256, 0, s.stream>>>(N, s.dim, s.x, s.xu[s.cur], s.v, s.mass, s.P, s.rp,
                                                   s.sell.row_of, s.sell.L, s.sell.slot_off, s.sell.col,
                                                   s.sell.coef, s.sell.word_off, s.sell.mask, t);
    MTS_LAUNCH_CHECK();
    double r[3];
    sum_rows(s, t, 3, N, r);
    s.arena.release(t);
    o->kinetic = r[0];
    o->strain_pd = r[1];
    o->external_work = r[2];
  }
  if (s.p.mode == MTS_COUPLED && s.nfe > 0) {
    double *t = s.arena.alloc<double>((size_t)2 * s.nfe);
    k_fe_node_terms<<<nb(s.nfe), 256, 0, s.stream>>>(s.nfe, s.dim, s.nact, s.uF, s.vF, s.mF, s.PF, t);
    MTS_LAUNCH_CHECK();
    double r[2];
    sum_rows(s, t, 2, s.nfe, r);
    s.arena.release(t);
    o->kinetic += r[0];
    o->external_work += r[1];
    fe_elem_forces_current(s);
    double *te = s.arena.alloc<double>((size_t)s.ne);
    k_fe_elem_terms<<<nb(s.ne), 256, 0, s.stream>>>(s.ne, s.nen, s.dim, s.conn, s.eact, s.uF, s.fe_buf, te);
    MTS_LAUNCH_CHECK();
    sum_rows(s, te, 1, s.ne, &o->strain_fe);
    s.arena.release(te);
  }
  o->n_broken = s.n_intact0 - count_intact(s);
}

}  // namespace mts
