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
#include <mutex>
#include <string>

#include "device_math.h"

namespace mts {

void fe_elem_forces_current(Solver &s);

namespace {

constexpr int kRed = 256;

// Fixed-order sum of the 256 values of a workgroup (value of thread t in
// v): a binary tree over LDS; the result is returned to thread 0.
__device__ inline double block_sum(double v, double *lds) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int h = kRed / 2; h > 0; h >>= 1) {
    if (t < h) lds[t] += lds[t + h];
    __syncthreads();
  }
  return lds[0];
}

// Per-workgroup partial sums over PD nodes: part[r * nblk + block] for row r =
// 0 kinetic, 1 PD deformation energy, 2 load work.
__global__ __launch_bounds__(kRed) void k_pd_energy_part(
    int64_t N, int dim, const double *x, const double *xu, const double *v, const double *mass, const double *Pf,
    const int32_t *rp, const int32_t *row_of, int L, const int64_t *slot_off, const int32_t *col,
    const double *coef, const int64_t *word_off, const uint64_t *mask, double *part, int64_t nblk) {
  __shared__ double lds[kRed];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double ek = 0.0, w = 0.0, e = 0.0;
  if (i < N) {
    double ui[3] = {0, 0, 0}, xi_[3] = {0, 0, 0};
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
    for (int k = 0; k < rp[i + 1] - rp[i]; k++) {
      if (!full_bit(word_off, mask, L, r, k)) continue;
      const int64_t pos = sell_slot(slot_off[sl], j, k, L);
      const int64_t c = col[pos];
      double xe = 0.0;
      for (int d = 0; d < dim; d++) xe += (x[d * N + c] - xi_[d]) * (xu[c * 2 * dim + dim + d] - ui[d]);
      e += coef[pos] * xe * xe;
    }
    e = 0.25 * e;
  }
  const double s0 = block_sum(ek, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s0;
  __syncthreads();
  const double s1 = block_sum(e, lds);
  if (threadIdx.x == 0) part[nblk + blockIdx.x] = s1;
  __syncthreads();
  const double s2 = block_sum(w, lds);
  if (threadIdx.x == 0) part[2 * nblk + blockIdx.x] = s2;
}

// Per-workgroup partial sums over FE nodes: row 0 kinetic, row 1 load work
// (active nodes only).
__global__ __launch_bounds__(kRed) void k_fe_node_part(int64_t nfe, int dim, const uint8_t *nact, const double *u,
                                                       const double *v, const double *m, const double *PF,
                                                       double *part, int64_t nblk) {
  __shared__ double lds[kRed];
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double ek = 0.0, w = 0.0;
  if (n < nfe && nact[n])
    for (int d = 0; d < dim; d++) {
      const double vd = v[n * dim + d];
      ek += 0.5 * m[n] * vd * vd;
      w += PF[n * dim + d] * u[n * dim + d];
    }
  const double s0 = block_sum(ek, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s0;
  __syncthreads();
  const double s1 = block_sum(w, lds);
  if (threadIdx.x == 0) part[nblk + blockIdx.x] = s1;
}

// Per-workgroup partial sums of 1/2 u_e . f_e over the active elements.
__global__ __launch_bounds__(kRed) void k_fe_elem_part(int64_t ne, int nen, int dim, const int32_t *conn,
                                                       const uint8_t *eact, const double *u, const double *fe_buf,
                                                       double *part) {
  __shared__ double lds[kRed];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (e < ne && eact[e]) {
    for (int a = 0; a < nen; a++)
      for (int d = 0; d < dim; d++) s += u[(int64_t)conn[e * nen + a] * dim + d] * fe_buf[(e * nen + a) * dim + d];
    s = 0.5 * s;
  }
  const double t = block_sum(s, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Per-workgroup counts of intact bonds: population count of the state words
// (padding bits are 0).
__global__ __launch_bounds__(kRed) void k_popcount_part(const uint64_t *w, int64_t n, double *part) {
  __shared__ double lds[kRed];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double c = i < n ? (double)__popcll(w[i]) : 0.0;
  const double t = block_sum(c, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// out[q] = sum of the n values of row q of terms, in a fixed order: thread t
// adds t, t + 256, ...; then a fixed tree.
__global__ __launch_bounds__(kRed) void k_sum_rows(const double *terms, int64_t n, double *out) {
  __shared__ double lds[kRed];
  const int t = threadIdx.x;
  const double *row = terms + blockIdx.x * n;
  double s = 0.0;
  for (int64_t i = t; i < n; i += kRed) s += row[i];
  const double r = block_sum(s, lds);
  if (t == 0) out[blockIdx.x] = r;
}

// Row sums res[0..6] (PD kinetic, PD deformation, PD load work, FE kinetic,
// FE load work, FE strain, intact bonds) into the five reported values.
__global__ void k_energy_combine(const double *res, int coupled, double n_intact0, double *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  out[0] = coupled ? res[0] + res[3] : res[0];
  out[1] = res[1];
  out[2] = coupled ? res[5] : 0.0;
  out[3] = coupled ? res[2] + res[4] : res[2];
  out[4] = n_intact0 - res[6];
}

inline int64_t nb(int64_t n) { return (n + kRed - 1) / kRed; }

// Partial sums the energy passes need at once (the largest phase).
int64_t energy_part_need(const Solver &s) {
  int64_t need = std::max<int64_t>(3 * nb(s.N), nb(std::max<int64_t>(s.sell.n_words, 1)));
  if (s.p.mode == MTS_COUPLED && s.nfe > 0) need = std::max(need, std::max(2 * nb(s.nfe), nb(s.ne)));
  return need;
}

// Enqueue the energy passes on the solver's stream: per-workgroup partial
// sums into part (energy_part_need doubles), their fixed-order row sums into
// res (7 doubles), and the five reported values (mts_energy_info order, the
// broken-bond count as a double) into out.  Launches kernels only.
void energy_enqueue(Solver &s, double *part, double *res, double *out) {
  hipStream_t st = s.stream;
  const int64_t N = s.N;
  const int64_t b = nb(N);
  k_pd_energy_part<<<(unsigned)b, kRed, 0, st>>>(N, s.dim, s.x, s.xu[s.cur], s.v, s.mass, s.P, s.rp, s.sell.row_of,
                                                  s.sell.L, s.sell.slot_off, s.sell.col, s.sell.coef,
                                                  s.sell.word_off, s.sell.mask, part, b);
  MTS_LAUNCH_CHECK();
  k_sum_rows<<<3, kRed, 0, st>>>(part, b, res);
  MTS_LAUNCH_CHECK();
  const bool coupled = s.p.mode == MTS_COUPLED && s.nfe > 0;
  if (coupled) {
    const int64_t bf = nb(s.nfe);
    k_fe_node_part<<<(unsigned)bf, kRed, 0, st>>>(s.nfe, s.dim, s.nact, s.uF, s.vF, s.mF, s.PF, part, bf);
    MTS_LAUNCH_CHECK();
    k_sum_rows<<<2, kRed, 0, st>>>(part, bf, res + 3);
    MTS_LAUNCH_CHECK();
    fe_elem_forces_current(s);
    const int64_t be = nb(s.ne);
    k_fe_elem_part<<<(unsigned)be, kRed, 0, st>>>(s.ne, s.nen, s.dim, s.conn, s.eact, s.uF, s.fe_buf, part);
    MTS_LAUNCH_CHECK();
    k_sum_rows<<<1, kRed, 0, st>>>(part, be, res + 5);
    MTS_LAUNCH_CHECK();
  }
  const int64_t nw = std::max<int64_t>(s.sell.n_words, 1);
  k_popcount_part<<<(unsigned)nb(nw), kRed, 0, st>>>(s.sell.mask, s.sell.n_words, part);
  MTS_LAUNCH_CHECK();
  k_sum_rows<<<1, kRed, 0, st>>>(part, nb(nw), res + 6);
  MTS_LAUNCH_CHECK();
  k_energy_combine<<<1, 64, 0, st>>>(res, coupled ? 1 : 0, (double)s.n_intact0, out);
  MTS_LAUNCH_CHECK();
}

// Static buffer of the energy variant that allocates nothing: the partial sums
// and row sums of one call.  Every GPU the library runs on holds its own copy
// until the process ends; calls on one GPU share it.
constexpr int64_t kNoAllocRes = 32;  // row sums (7 used), then the partial sums
constexpr int64_t kNoAllocDoubles = (int64_t)1 << 16;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current.
double *scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw ArgError{"device ordinal out of range"};
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int prev = -1;
    MTS_HIP(hipGetDevice(&prev));
    if (prev != dev) MTS_HIP(hipSetDevice(dev));
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (prev != dev) MTS_HIP(hipSetDevice(prev));
    MTS_HIP(e);
    if (!ptr) throw HipError{hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__};
    g_scratch_ptr[dev] = static_cast<double *>(ptr);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

int64_t count_intact(Solver &s) {
  const int64_t n = std::max<int64_t>(s.sell.n_words, 1);
  double *part = s.arena.alloc<double>((size_t)nb(n));
  double *dout = s.arena.alloc<double>(1);
  k_popcount_part<<<(unsigned)nb(n), kRed, 0, s.stream>>>(s.sell.mask, s.sell.n_words, part);
  MTS_LAUNCH_CHECK();
  k_sum_rows<<<1, kRed, 0, s.stream>>>(part, nb(n), dout);
  MTS_LAUNCH_CHECK();
  double c = 0.0;
  MTS_HIP(hipMemcpyAsync(&c, dout, sizeof(double), hipMemcpyDeviceToHost, s.stream));
  MTS_HIP(hipStreamSynchronize(s.stream));
  s.arena.release(part);
  s.arena.release(dout);
  return (int64_t)c;
}

void energy_impl(Solver &s, mts_energy_info *o) {
  std::memset(o, 0, sizeof *o);
  double *part = s.arena.alloc<double>((size_t)energy_part_need(s));
  double *res = s.arena.alloc<double>(16);
  double *out = res + 8;
  energy_enqueue(s, part, res, out);
  double h[5];
  MTS_HIP(hipMemcpyAsync(h, out, sizeof h, hipMemcpyDeviceToHost, s.stream));
  MTS_HIP(hipStreamSynchronize(s.stream));
  s.arena.release(part);
  s.arena.release(res);
  o->kinetic = h[0];
  o->strain_pd = h[1];
  o->strain_fe = h[2];
  o->external_work = h[3];
  o->n_broken = (int64_t)h[4];
}

// The same passes with the partial sums in the static buffer: no allocation,
// kernels only, results into caller device memory.
void energy_noalloc_impl(Solver &s, double *dev_out) {
  const int64_t need = energy_part_need(s);
  if (need > kNoAllocDoubles - kNoAllocRes)
    throw ArgError{"mts_energy_noalloc: the solver needs " + std::to_string(need) +
                   " partial sums; the static buffer holds " + std::to_string(kNoAllocDoubles - kNoAllocRes) +
                   " (about " + std::to_string((kNoAllocDoubles - kNoAllocRes) / 3 * kRed) + " PD nodes)"};
  double *base = scratch_address(s.device);
  energy_enqueue(s, base + kNoAllocRes, base, dev_out);
}

}  // namespace mts
