// C-ABI of the mtspd library: problem validation, solver construction, the
// macro-step driver (Algorithm 1), state access and per-kernel timing.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.h"

#include <chrono>
#include <cstdarg>
#include <cstdlib>

namespace mts {

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void vlog(const Solver &s, const char *fmt, ...) {
  if (!s.verbose) return;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "[mtspd %8.3f s] %s\n", now_s() - s.t_create0, buf);
  std::fflush(stderr);
}

void DeviceArena::release(void *p) {
  if (region) {
    auto it = used_ext.find((size_t)(static_cast<char *>(p) - region));
    if (it == used_ext.end()) return;
    size_t off = it->first, sz = it->second;
    used_ext.erase(it);
    live -= sz;
    auto nx = free_ext.lower_bound(off);
    if (nx != free_ext.end() && nx->first == off + sz) {  // merge with the next free extent
      sz += nx->second;
      nx = free_ext.erase(nx);
    }
    if (nx != free_ext.begin()) {  // and with the previous one
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        pv->second += sz;
        return;
      }
    }
    free_ext[off] = sz;
    return;
  }
  for (size_t k = 0; k < blocks.size(); k++)
    if (blocks[k].first == p) {
      (void)hipFree(p);
      live -= blocks[k].second;
      blocks.erase(blocks.begin() + (long)k);
      return;
    }
}

void DeviceArena::free_all() {
  for (auto &b : blocks) (void)hipFree(b.first);
  blocks.clear();
  live = 0;
  if (region) use_region(region, region_bytes);  // the region itself stays the caller's
}

void Solver::prof_begin(int k, hipEvent_t *e0) {
  *e0 = nullptr;
  if (!profiling) return;
  hipEvent_t e;
  if (!ev_pool.empty()) {
    e = ev_pool.back();
    ev_pool.pop_back();
  } else {
    MTS_HIP(hipEventCreate(&e));
  }
  MTS_HIP(hipEventRecord(e, stream));
  *e0 = e;
  (void)k;
}

void Solver::prof_end(int k, hipEvent_t e0, int launches) {
  if (!profiling || !e0) return;
  hipEvent_t e;
  if (!ev_pool.empty()) {
    e = ev_pool.back();
    ev_pool.pop_back();
  } else {
    MTS_HIP(hipEventCreate(&e));
  }
  MTS_HIP(hipEventRecord(e, stream));
  ev_pending[k].push_back({e0, e, launches});
}

void Solver::prof_collect() {
  for (int k = 0; k < MTS_KT_COUNT; k++) {
    for (auto &pr : ev_pending[k]) {
      MTS_HIP(hipEventSynchronize(pr.e1));
      float ms = 0.f;
      MTS_HIP(hipEventElapsedTime(&ms, pr.e0, pr.e1));
      kt_ms[k] += ms;
      kt_count[k] += pr.launches;
      ev_pool.push_back(pr.e0);
      ev_pool.push_back(pr.e1);
    }
    ev_pending[k].clear();
  }
}

namespace {

thread_local char g_err[1024];

// int_0^delta r^n exp(-r/l) dr in closed form.
double exp_moment(int n, double delta, double l) {
  double t = delta / l, term = 1.0, sum = 1.0, fact = 1.0;
  for (int k = 1; k <= n; k++) {
    term = term * t / (double)k;
    sum = sum + term;
    fact = fact * (double)k;
  }
  return std::pow(l, (double)(n + 1)) * fact * (1.0 - std::exp(-t) * sum);
}

void validate(const mts_problem *p) {
  if (!p) throw ArgError{"null problem"};
  if (p->dim != 2 && p->dim != 3) throw ArgError{"dim must be 2 or 3"};
  if (p->mode != MTS_COUPLED && p->mode != MTS_PURE_PD) throw ArgError{"unknown mode"};
  if (p->precision != MTS_FP64 && p->precision != MTS_MIXED) throw ArgError{"unknown precision"};
  if (p->m < 1) throw ArgError{"m must be >= 1"};
  if (!(p->dt_pd > 0.0) || !std::isfinite(p->dt_pd)) throw ArgError{"dt_pd must be > 0"};
  if (!(p->horizon_factor >= 1.0)) throw ArgError{"horizon_factor must be >= 1"};
  if (!(p->dx > 0.0)) throw ArgError{"dx must be > 0"};
  if (p->n_pd <= 0 || !p->host_pd_pos) throw ArgError{"no PD nodes"};
  if (p->n_pd >= ((int64_t)1 << 31)) throw ArgError{"too many PD nodes"};
  if (p->n_cracks < 0 || p->n_cracks > 8) throw ArgError{"n_cracks must be 0..8"};
  if (p->dim == 3 && p->n_cracks > 0) throw ArgError{"cracks are supported in 2D only"};
  if (!(p->E > 0.0) || !(p->rho > 0.0) || !(p->thickness > 0.0)) throw ArgError{"E, rho, thickness must be > 0"};
  if (!(p->s_crit > 0.0) && !(p->G0 > 0.0)) throw ArgError{"need s_crit > 0 or G0 > 0"};
  if (p->kernel != MTS_K_PMB && p->kernel != MTS_K_EXP) throw ArgError{"unknown kernel"};
  if (p->kernel == MTS_K_EXP && !(p->l_over_delta > 0.0)) throw ArgError{"l_over_delta must be > 0"};
  if (p->mode == MTS_COUPLED) {
    for (int a = 0; a < p->dim; a++)
      if (p->fe_n[a] < 1) throw ArgError{"coupled mode needs fe_n >= 1 on every axis"};
    if (!(p->fe_h > 0.0) || !(p->overlap > 0.0)) throw ArgError{"coupled mode needs fe_h > 0 and overlap > 0"};
    if (p->weight_kind < 0 || p->weight_kind > 2) throw ArgError{"unknown weight_kind"};
  }
  if (!(p->fe_beta == 0.0 || p->fe_beta == 0.25)) throw ArgError{"fe_beta must be 0 (explicit) or 1/4"};
  if (!std::isfinite(p->traction_x)) throw ArgError{"non-finite traction_x"};
  if (p->clamp_x0 != 0 && p->clamp_x0 != 1) throw ArgError{"clamp_x0 must be 0 or 1"};
  if (p->mode != MTS_COUPLED && (p->traction_x != 0.0 || p->clamp_x0))
    throw ArgError{"traction_x and clamp_x0 act on the FE mesh (coupled mode)"};
  if (p->clamp_x0 && p->vel_bc != 0.0) throw ArgError{"clamp_x0 needs vel_bc = 0"};
  if (!(p->pd_beta == 0.0 || p->pd_beta == 0.25)) throw ArgError{"pd_beta must be 0 (explicit) or 1/4"};
  if (p->pd_beta != 0.0 && (p->mode != MTS_PURE_PD || p->precision != MTS_FP64))
    throw ArgError{"the implicit PD step runs in pure-PD mode and FP64"};
  for (int64_t i = 0; i < p->n_pd * p->dim; i++)
    if (!std::isfinite(p->host_pd_pos[i])) throw ArgError{"non-finite node position"};
}

// Scalar parameters of the method (Eq. 2 calibration, critical stretch, steps).
void derive_params(Solver &s) {
  const mts_problem &p = s.p;
  Params &P = s.prm;
  const double pi = 3.14159265358979323846;
  P.dim = p.dim;
  P.weight_kind = p.weight_kind;
  P.kernel = p.kernel;
  P.coupled = p.mode == MTS_COUPLED ? 1 : 0;
  P.delta = p.horizon_factor * p.dx;
  P.d2 = P.delta * P.delta;
  P.V = p.dim == 2 ? p.dx * p.dx * p.thickness : p.dx * p.dx * p.dx;
  P.VV = P.V * P.V;
  const double dl = P.delta, E = p.E;
  double I6, I7;
  if (p.kernel == MTS_K_EXP) {
    P.lexp = dl * p.l_over_delta;
    P.c0 = p.dim == 2 ? 3.0 * E / (pi * p.thickness * exp_moment(5, dl, P.lexp))
                      : 3.0 * E / (pi * exp_moment(6, dl, P.lexp));
    I6 = P.c0 * exp_moment(6, dl, P.lexp);
    I7 = P.c0 * exp_moment(7, dl, P.lexp);
  } else {
    P.lexp = 1.0;
    P.c0 = p.dim == 2 ? 9.0 * E / (pi * p.thickness * dl * dl * dl) : 12.0 * E / (pi * dl * dl * dl * dl);
    I6 = P.c0 * dl * dl * dl * dl / 4.0;
    I7 = P.c0 * dl * dl * dl * dl * dl / 5.0;
  }
  if (p.s_crit > 0.0) P.scrit = p.s_crit;
  else if (p.dim == 2) P.scrit = std::sqrt(p.G0 / (p.thickness * I6));
  else P.scrit = std::sqrt(2.0 * p.G0 / (pi * I7));
  P.K2 = (1.0 + P.scrit) * (1.0 + P.scrit);
  P.K2m1f = (float)(2.0 * P.scrit + P.scrit * P.scrit);
  P.dtP = p.dt_pd;
  P.hdtP = 0.5 * P.dtP;
  P.hdt2P = 0.5 * P.dtP * P.dtP;
  P.dtF = (double)p.m * P.dtP;
  P.hdtF = 0.5 * P.dtF;
  P.hdt2F = 0.5 * P.dtF * P.dtF;
  for (int a = 0; a < 3; a++) {
    P.o2lo[a] = 0.0;
    P.o2hi[a] = 0.0;
  }
  for (int a = 0; a < p.dim; a++) {
    double tol = 1e-9 * (p.dom_hi[a] - p.dom_lo[a]);
    P.o2lo[a] = p.pd_lo[a] + (std::fabs(p.pd_lo[a] - p.dom_lo[a]) > tol ? p.overlap : 0.0);
    P.o2hi[a] = p.pd_hi[a] - (std::fabs(p.pd_hi[a] - p.dom_hi[a]) > tol ? p.overlap : 0.0);
  }
  P.overlap = p.overlap;
  P.rho = p.rho;
}

}  // namespace

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

void create_impl(const mts_problem *pin, void *stream, Solver *s) {
  validate(pin);
  MTS_HIP(hipGetDevice(&s->device));
  s->verbose = std::getenv("MTS_VERBOSE") != nullptr;
  if (const char *t = std::getenv("MTS_TILE")) s->tiled = std::atoi(t) != 0 ? 1 : 0;  // tuning: row order
  if (const char *t = std::getenv("MTS_PD_VARIANT")) s->pd_variant = std::atoi(t);  // tuning: loop shape
  if (const char *t = std::getenv("MTS_HALO")) s->halo = std::atoi(t) != 0;          // tuning: LDS staging
  if (const char *t = std::getenv("MTS_REGION_LANES")) {  // tuning: link region lanes per row
    const int v = std::atoi(t);
    s->region_lanes = (v == 1 || v == 2 || v == 4 || v == 8) ? v : 0;
  }
  if (const char *t = std::getenv("MTS_HALO_WAVES")) s->halo_waves = std::atoi(t) == 8 ? 8 : 4;  // tuning
  if (const char *t = std::getenv("MTS_SUBCYCLE")) s->subcycle = std::atoi(t) != 0;  // one launch per macro step
  if (const char *t = std::getenv("MTS_INV_DROP")) s->sym.prune = std::atoi(t) != 0;  // tests: read every tile
  if (const char *t = std::getenv("MTS_FULL_REBUILD")) s->incremental = std::atoi(t) == 0;  // tests: every column
  if (const char *t = std::getenv("MTS_SYM_FORM")) s->sym.form = std::min(std::max(std::atoi(t), 0), 2);  // tests
  if (const char *t = std::getenv("MTS_BUILD_STREAMS"))  // tests: fewer streams for a build's colour batches
    s->build_streams = std::min(std::max(std::atoi(t), 1), s->build_streams);
  if (const char *t = std::getenv("MTS_SPIN_LIMIT")) s->spin_limit = (uint32_t)std::strtoul(t, nullptr, 10);  // tests
  const char *e = s->force_lanes ? nullptr : std::getenv("MTS_LANES");
  if (e) {  // tuning: lanes per row of the bond pass
    const int L = std::atoi(e);
    if (L == 1 || L == 2 || L == 4 || L == 8) s->force_lanes = L;
  }
  s->t_create0 = now_s();
  s->p = *pin;
  const int dim = s->dim = pin->dim;
  const int64_t N = s->N = pin->n_pd;
  s->pos.assign(pin->host_pd_pos, pin->host_pd_pos + N * dim);
  s->p.host_pd_pos = nullptr;
  s->stream = (hipStream_t)stream;
  s->precision = pin->precision;
  s->breaking = pin->breaking != 0;
  s->m = pin->m;
  s->fe_beta = pin->mode == MTS_COUPLED ? pin->fe_beta : 0.0;
  s->pd_beta = pin->pd_beta;
  derive_params(*s);
  DeviceArena &ar = s->arena;
  hipStream_t st = s->stream;
  // positions, SoA
  s->x = ar.alloc<double>((size_t)dim * N);
  {
    std::vector<double> soa((size_t)dim * N);
    for (int64_t i = 0; i < N; i++)
      for (int d = 0; d < dim; d++) soa[(size_t)d * N + i] = s->pos[(size_t)i * dim + d];
    MTS_HIP(hipMemcpyAsync(s->x, soa.data(), sizeof(double) * dim * N, hipMemcpyHostToDevice, st));
    MTS_HIP(hipStreamSynchronize(st));
  }
  s->alpha = ar.alloc<double>(N);
  s->mass = ar.alloc<double>(N);
  s->xu[0] = ar.alloc<double>((size_t)2 * dim * N);
  s->xu[1] = ar.alloc<double>((size_t)2 * dim * N);
  {
    std::vector<double> rec((size_t)2 * dim * N, 0.0);
    for (int64_t i = 0; i < N; i++)
      for (int d = 0; d < dim; d++) rec[(size_t)i * 2 * dim + d] = s->pos[(size_t)i * dim + d];
    for (double *q : s->xu)
      MTS_HIP(hipMemcpyAsync(q, rec.data(), sizeof(double) * rec.size(), hipMemcpyHostToDevice, st));
    MTS_HIP(hipStreamSynchronize(st));
  }
  s->v = ar.alloc<double>((size_t)dim * N);
  s->a = ar.alloc<double>((size_t)dim * N);
  s->damage = ar.alloc<double>(N);
  for (double *q : {s->v, s->a}) MTS_HIP(hipMemsetAsync(q, 0, sizeof(double) * dim * N, st));
  MTS_HIP(hipMemsetAsync(s->damage, 0, sizeof(double) * N, st));
  s->region_flag = ar.alloc<int32_t>(1);
  MTS_HIP(hipMemsetAsync(s->region_flag, 0, sizeof(int32_t), st));
  s->nonfinite_flag = ar.alloc<int32_t>(2);
  MTS_HIP(hipMemsetAsync(s->nonfinite_flag, 0, 2 * sizeof(int32_t), st));
  MTS_HIP(hipEventCreateWithFlags(&s->nf_event, hipEventDisableTiming));
  build_neighbors(*s);
  vlog(*s, "neighbours: %lld nodes, %lld bonds, %d lanes per row", (long long)N, (long long)s->nnz, s->sell.L);
  pd_setup(*s);
  pd_implicit_setup(*s);
  if (pin->mode == MTS_COUPLED) {
    fe_setup(*s);
    vlog(*s, "fe: %lld nodes, %lld elements", (long long)s->nfe, (long long)s->ne);
    coupling_setup(*s);
  }
  pd_predict_all(*s);
  MTS_HIP(hipHostMalloc((void **)&s->pinned_flag, 4 * sizeof(int32_t), hipHostMallocDefault));
  s->pinned_flag[0] = s->pinned_flag[1] = s->pinned_flag[2] = s->pinned_flag[3] = 0;
  pd_damage(*s);
  s->n_intact0 = count_intact(*s);
  MTS_HIP(hipStreamSynchronize(st));
}

mts_status fail_from_exception() {
  try {
    throw;
  } catch (const HipError &e) {
    std::snprintf(g_err, sizeof g_err, "HIP error %d (%s) in %s at %s:%d", (int)e.err, hipGetErrorString(e.err),
                  e.expr, e.file, e.line);
    return MTS_EDEVICE;
  } catch (const ArgError &e) {
    std::snprintf(g_err, sizeof g_err, "%s", e.msg.c_str());
    return MTS_EINVAL;
  } catch (const MemError &e) {
    std::snprintf(g_err, sizeof g_err, "%s", e.msg.c_str());
    return MTS_ENOMEM;
  } catch (const std::bad_alloc &) {
    std::snprintf(g_err, sizeof g_err, "host allocation failed");
    return MTS_ENOMEM;
  } catch (...) {
    std::snprintf(g_err, sizeof g_err, "unexpected internal error");
    return MTS_EDEVICE;
  }
}

__global__ void k_soa_to_aos(const double *src, double *dst, int64_t N, int dim) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  for (int d = 0; d < dim; d++) dst[i * dim + d] = src[(int64_t)d * N + i];
}

__global__ void k_aos_to_soa(const double *src, double *dst, int64_t N, int dim) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  for (int d = 0; d < dim; d++) dst[(int64_t)d * N + i] = src[i * dim + d];
}

// displacement part of the node records <-> node-major vectors
__global__ void k_xu_to_aos(const double *xu, double *dst, int64_t N, int dim) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  for (int d = 0; d < dim; d++) dst[i * dim + d] = xu[i * 2 * dim + dim + d];
}

__global__ void k_aos_to_xu(const double *src, double *xu, int64_t N, int dim) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  for (int d = 0; d < dim; d++) xu[i * 2 * dim + dim + d] = src[i * dim + d];
}

__global__ void k_nonfinite(const double *a, int64_t n, int32_t *flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(a[i])) flag[0] = 1;
}

void check_finite(Solver &s) {
  int32_t *f = s.arena.alloc<int32_t>(1);
  MTS_HIP(hipMemsetAsync(f, 0, sizeof(int32_t), s.stream));
  int64_t n = (int64_t)s.dim * s.N;
  k_nonfinite<<<(unsigned)((n + 255) / 256), 256, 0, s.stream>>>(s.v, n, f);
  MTS_LAUNCH_CHECK();
  int32_t h = 0;
  MTS_HIP(hipMemcpyAsync(&h, f, sizeof(int32_t), hipMemcpyDeviceToHost, s.stream));
  MTS_HIP(hipStreamSynchronize(s.stream));
  s.arena.release(f);
  if (h) s.unstable = true;
}

__global__ void k_snapshot(const uint64_t *mask, uint64_t *snap, int64_t n, int32_t *flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) snap[i] = mask[i];
  if (i == 0) flag[0] = 0;
}

// Save the bond states of this macro step and move its rebuild flag to the
// host (the copy is ordered before the kernel that clears the device flag; no
// memset, so the sequence can be recorded into a graph).
void snapshot_states(Solver &s, int slot) {
  MTS_HIP(hipMemcpyAsync(s.pinned_flag + slot, s.region_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s.stream));
  snapshot_masks(s, slot);
}

void snapshot_masks(Solver &s, int slot) {
  const int64_t n = std::max<int64_t>(s.sell.n_words, 1);
  k_snapshot<<<(unsigned)((n + 255) / 256), 256, 0, s.stream>>>(s.sell.mask, s.mask_snap[slot], s.sell.n_words,
                                                               s.region_flag);
  MTS_LAUNCH_CHECK();
}

// Algorithm 1, last step: the unit-load responses are rebuilt after a macro step
// in which a bond inside their support broke.  The check for step k-1 is
// resolved after step k's free problem has been enqueued (it does not use the
// responses), so the host wait overlaps device work; the rebuild uses the bond
// states saved at the end of step k-1, exactly as if it had run right then.
void resolve_pending(Solver &s) {
  if (!s.pending) return;
  const int slot = s.pending_slot;
  MTS_HIP(hipEventSynchronize(s.flag_event[slot]));
  s.pending = false;
  if (s.pinned_flag[3]) s.wait_gave_up = true;
  if (s.pinned_flag[2] || s.pinned_flag[3]) {  // a velocity of that macro step was not finite: stop here
    s.unstable = s.unstable || s.pinned_flag[2] != 0;
    return;
  }
  if (s.pinned_flag[slot]) {
    s.pinned_flag[slot] = 0;
    hipEvent_t e0;
    s.prof_begin(MTS_KT_REBUILD, &e0);
    coupling_rebuild(s, s.mask_snap[slot]);
    s.prof_end(MTS_KT_REBUILD, e0);
    s.n_rebuilds++;
  }
}

// The non-finite flag of the last macro step of an earlier mts_advance call,
// when its copy to the host has completed (no wait).
void poll_nonfinite(Solver &s) {
  if (!s.nf_recorded) return;
  const hipError_t q = hipEventQuery(s.nf_event);
  if (q == hipErrorNotReady) return;
  MTS_HIP(q);
  if (s.pinned_flag[2]) s.unstable = true;
  if (s.pinned_flag[3]) s.wait_gave_up = true;
}

void advance_impl(Solver &s, int64_t n) {
  const bool coupled = s.p.mode == MTS_COUPLED;
  const bool track = coupled && s.m >= 2;
  poll_nonfinite(s);
  for (int64_t k = 0; k < n && !s.unstable && !s.wait_gave_up; k++) {
    if (coupled && !s.fe_free_done) {
      hipEvent_t e0 = nullptr;
      s.prof_begin(MTS_KT_FE, &e0);
      fe_free_step(s);
      s.prof_end(MTS_KT_FE, e0);
    }
    s.fe_free_done = false;
    {
      // the m substep launches run back to back; one event pair brackets them
      hipEvent_t e0 = nullptr;
      s.prof_begin(MTS_KT_PD_SUBSTEP, &e0);
      if (s.pd_beta > 0.0) {
        for (int j = 1; j <= s.m; j++) pd_implicit_step(s);
      } else if (!pd_subcycle(s)) {
        for (int j = 1; j <= s.m; j++) pd_substep(s, j);
      }
      s.prof_end(MTS_KT_PD_SUBSTEP, e0, s.m);
    }
    int slot = -1;
    if (track) {
      // the rebuild flag goes to the host now; the bond states are saved (and
      // the flag cleared) by extra workgroups of a link launch below, before
      // the next macro step's substeps and any rebuild that reads them
      slot = (int)(s.macro_steps & 1);
      MTS_HIP(hipMemcpyAsync(s.pinned_flag + slot, s.region_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s.stream));
      MTS_HIP(hipMemcpyAsync(s.pinned_flag + 2, s.nonfinite_flag, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s.stream));
      MTS_HIP(hipEventRecord(s.flag_event[slot], s.stream));
    }
    resolve_pending(s);  // previous macro step's check
    if (s.unstable || s.wait_gave_up) break;
    // the next macro step's FE free step joins this one's link launches when
    // another macro step of this call follows (the state between calls stays
    // that of a whole macro step) and no per-phase timing is taken
    if (coupled) s.fe_free_done = coupling_solve_and_correct(s, k + 1 < n && !s.profiling && s.fe_beta == 0.0, slot);
    if (track) {
      s.pending = true;
      s.pending_slot = slot;
    }
    s.macro_steps++;
  }
  if (!s.unstable && !s.wait_gave_up && n > 0) {
    MTS_HIP(hipMemcpyAsync(s.pinned_flag + 2, s.nonfinite_flag, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s.stream));
    MTS_HIP(hipEventRecord(s.nf_event, s.stream));
    s.nf_recorded = true;
  }
}

int64_t qsize(Solver &s, int what) {
  switch (what) {
    case MTS_PD_U: case MTS_PD_V: case MTS_PD_A: return s.N * s.dim;
    case MTS_FE_U: case MTS_FE_V: case MTS_FE_A: case MTS_FE_X: return s.nfe * s.dim;
    case MTS_DAMAGE: case MTS_PD_ALPHA: case MTS_PD_MASS: return s.N;
    case MTS_LAMBDA: return s.nl;
    case MTS_FE_MASS: return s.nfe;
    case MTS_CONSTRAINT_NODES: return s.nc;
    case MTS_H: return s.Hcopy ? s.nl * s.nl : -1;
    default: return -1;
  }
}

}  // namespace mts

using namespace mts;

struct mts_solver {
  Solver s;
};

extern "C" {

const char *mts_last_error(void) { return g_err; }

const char *mts_status_str(mts_status st) {
  switch (st) {
    case MTS_OK: return "ok";
    case MTS_EINVAL: return "invalid argument";
    case MTS_ENOMEM: return "out of memory";
    case MTS_EDEVICE: return "device error";
    case MTS_EUNSTABLE: return "unstable (non-finite state)";
    case MTS_EAGAIN: return "try again";
    case MTS_ETOOBIG: return "request too big";
    case MTS_ESTATE: return "invalid state";
  }
  return "unknown status";
}

mts_status mts_plan(const mts_problem *p, mts_plan_info *out) {
  try {
    if (!out) throw ArgError{"null output"};
    validate(p);
    std::memset(out, 0, sizeof *out);
    const double hf = p->horizon_factor;
    // lattice family size for this horizon (upper estimate for near-lattice inputs)
    int64_t fam = 0;
    int r = (int)std::floor(hf + 0.01);
    for (int c = (p->dim == 3 ? -r : 0); c <= (p->dim == 3 ? r : 0); c++)
      for (int b = -r; b <= r; b++)
        for (int a = -r; a <= r; a++)
          if ((a || b || c) && (double)(a * a + b * b + c * c) <= (hf + 0.01) * (hf + 0.01)) fam++;
    out->n_pd = p->n_pd;
    out->nnz_estimate = p->n_pd * fam;
    int64_t nfe = 0, ne = 0;
    if (p->mode == MTS_COUPLED) {
      nfe = (int64_t)(p->fe_n[0] + 1) * (p->fe_n[1] + 1) * (p->dim == 3 ? p->fe_n[2] + 1 : 1);
      ne = (int64_t)p->fe_n[0] * p->fe_n[1] * (p->dim == 3 ? p->fe_n[2] : 1);
      nfe += p->fe_n[0] + 1;
    }
    out->n_fe_nodes = nfe;
    // constraint estimate: nodes within `overlap` of the PD box faces
    int64_t nc = 0;
    if (p->mode == MTS_COUPLED) {
      double vol_in = 1.0, vol = 1.0;
      for (int a = 0; a < p->dim; a++) {  // bands only on the faces inside the domain
        const double L = p->pd_hi[a] - p->pd_lo[a], tol = 1e-9 * (p->dom_hi[a] - p->dom_lo[a]);
        const int inner = (p->pd_lo[a] > p->dom_lo[a] + tol) + (p->pd_hi[a] < p->dom_hi[a] - tol);
        vol *= L;
        vol_in *= std::max(0.0, L - inner * p->overlap);
      }
      nc = (int64_t)std::ceil(p->n_pd * (1.0 - vol_in / vol)) + 64;
    }
    out->n_constraints_estimate = nc;
    // An upper estimate of everything the solver allocates during mts_create
    // (temporaries included, as if none were freed), used for pool admission
    // and to size a caller arena.
    const int64_t nl = nc * p->dim, d = p->dim;
    const int64_t rhs = d == 2 ? 8 : 6;
    const int64_t slots = out->nnz_estimate + out->nnz_estimate / 10 + p->n_pd;  // sliced-ELL padding
    // per slot: index 4, coefficients 8 + 4, slot record 12, state bit, staging
    // index 4 (temporary), canonical CSR index 4; per node: positions, records,
    // velocities, accelerations, loads, weights, masses, damage, maps, cell lists
    int64_t bytes = slots * 40 + p->n_pd * (96 * d + 96) + ((int64_t)8 << 20);
    if (p->mode == MTS_COUPLED) {
      const int64_t T = (nl + 63) / 64, tiles = T * (T + 1) / 2;
      bytes += nl * nl * 8 * (nl <= 4096 ? 2 : 1);   // H (and its copy, when kept)
      bytes += tiles * (64 * 64 * 8 + 2 * 64 * 8 + 32);  // packed inverse, GEMV partial sums, tile lists
      bytes += T * 64 * 8 + nl * 12 + T * 64;         // right-hand side in both orders, the map, reduction lists
      bytes += 2 * T * 64 * 256 * 8 + 256 * 256 * 8 + 64 * 64 * 8;  // sweep panels and pivot blocks
      // link responses (one set per build stream), final-update records
      bytes += Solver::kBuildStreams * (4 * rhs * d * p->n_pd * 8 + p->n_pd * 4) + 2 * 2 * d * p->n_pd * 8;
      bytes += slots * 40;                            // link region layout (at most every slot)
      bytes += ne * 8 * 8 * 8 + nfe * 8 * 24 + nc * 64 * 8;  // FE mesh and state, coupling tables
      bytes += slots / 8 + p->n_pd + nc * 8;          // last build's bond states, changed-node and column flags
    }
    bytes += bytes / 8;
    out->device_bytes_estimate = bytes;
    return MTS_OK;
  } catch (...) {
    return fail_from_exception();
  }
}

mts_status mts_create(const mts_problem *p, void *hip_stream, mts_solver **out) {
  return mts_create_in(p, nullptr, 0, hip_stream, out);
}

mts_status mts_create_in(const mts_problem *p, void *dev_arena, int64_t arena_bytes, void *hip_stream,
                         mts_solver **out) {
  if (!out) {
    std::snprintf(g_err, sizeof g_err, "null output pointer");
    return MTS_EINVAL;
  }
  *out = nullptr;
  if (dev_arena && (arena_bytes <= 0 || ((uintptr_t)dev_arena & 255u) != 0)) {
    std::snprintf(g_err, sizeof g_err, "the arena must be 256-byte aligned and non-empty");
    return MTS_EINVAL;
  }
  mts_solver *h = nullptr;
  try {
    h = new mts_solver();
    if (dev_arena) h->s.arena.use_region(dev_arena, (size_t)arena_bytes);
    create_impl(p, hip_stream, &h->s);
    *out = h;
    return MTS_OK;
  } catch (...) {
    mts_status st = fail_from_exception();
    if (h) {
      (void)hipStreamSynchronize(h->s.stream);
      (void)hipGetLastError();
      if (h->s.pinned_flag) (void)hipHostFree(h->s.pinned_flag);
      if (h->s.nf_event) (void)hipEventDestroy(h->s.nf_event);
      coupling_free(h->s);
      fe_implicit_free(h->s);
      pd_implicit_free(h->s);
      h->s.arena.free_all();
      delete h;
    }
    return st;
  }
}

mts_status mts_advance(mts_solver *h, int64_t n) {
  if (!h) return (std::snprintf(g_err, sizeof g_err, "null solver"), MTS_EINVAL);
  if (n < 0) return (std::snprintf(g_err, sizeof g_err, "negative step count"), MTS_EINVAL);
  if (h->s.unstable) return (std::snprintf(g_err, sizeof g_err, "solver is unstable"), MTS_EUNSTABLE);
  if (h->s.wait_gave_up)
    return (std::snprintf(g_err, sizeof g_err, "a bounded wait of the subcycle kernel gave up"), MTS_EDEVICE);
  try {
    advance_impl(h->s, n);
    if (h->s.wait_gave_up) {
      std::snprintf(g_err, sizeof g_err, "a bounded wait of the subcycle kernel gave up (%lld macro steps enqueued)",
                    (long long)h->s.macro_steps);
      return MTS_EDEVICE;
    }
    if (h->s.unstable) {
      std::snprintf(g_err, sizeof g_err, "non-finite PD velocity at the end of a macro step (%lld macro steps enqueued)",
                    (long long)h->s.macro_steps);
      return MTS_EUNSTABLE;
    }
    return MTS_OK;
  } catch (...) {
    return fail_from_exception();
  }
}

mts_status mts_sync(mts_solver *h) {
  if (!h) return (std::snprintf(g_err, sizeof g_err, "null solver"), MTS_EINVAL);
  try {
    resolve_pending(h->s);
    MTS_HIP(hipStreamSynchronize(h->s.stream));
    if (h->s.pinned_flag[2]) h->s.unstable = true;
    if (h->s.pinned_flag[3]) h->s.wait_gave_up = true;
    if (h->s.wait_gave_up) {
      std::snprintf(g_err, sizeof g_err, "a bounded wait of the subcycle kernel gave up");
      return MTS_EDEVICE;
    }
    check_finite(h->s);
    if (h->s.unstable) {
      std::snprintf(g_err, sizeof g_err, "non-finite PD velocity");
      return MTS_EUNSTABLE;
    }
    return MTS_OK;
  } catch (...) {
    return fail_from_exception();
  }
}

mts_status mts_read(mts_solver *h, int32_t what, double *out, int64_t cap, int64_t *n) {
  if (!h || !out) return (std::snprintf(g_err, sizeof g_err, "null argument"), MTS_EINVAL);
  return read_impl(h->s, what, out, cap, n);
}

mts_status mts_energy(mts_solver *h, mts_energy_info *out) {
  if (!h || !out) return (std::snprintf(g_err, sizeof g_err, "null argument"), MTS_EINVAL);
  try {
    energy_impl(h->s, out);
    return MTS_OK;
  } catch (...) {
    return fail_from_exception();
  }
}

mts_status mts_energy_noalloc(mts_solver *h, double *dev_out) {
  if (!h || !dev_out) return (std::snprintf(g_err, sizeof g_err, "null argument"), MTS_EINVAL);
  try {
    energy_noalloc_impl(h->s, dev_out);
    return MTS_OK;
  } catch (...) {
    return fail_from_exception();
  }
}

mts_status mts_read_device(mts_solver *h, int32_t what, double *dev_out, int64_t cap, int64_t *n) {
  if (!h || !dev_out) return (std::snprintf(g_err, sizeof g_err, "null argument"), MTS_EINVAL);
  return read_device_impl(h->s, what, dev_out, cap, n);
}

}  // extern "C"

namespace mts {
namespace {
__global__ void k_index_to_double(const int32_t *a, int64_t n, double *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)a[i];
}
}  // namespace

// Device-side read: the node-major form of a quantity written into dev_out on
// the solver's stream (no host synchronization).
mts_status read_device_impl(Solver &s, int32_t what, double *dev_out, int64_t cap, int64_t *n) {
  try {
    const int64_t sz = qsize(s, what);
    if (sz < 0) throw ArgError{"quantity not available"};
    if (cap < sz) throw ArgError{"output capacity too small"};
    if (n) *n = sz;
    if (sz == 0) return MTS_OK;
    hipStream_t st = s.stream;
    const unsigned nb = (unsigned)((s.N + 255) / 256);
    const double *src = nullptr;
    switch (what) {
      case MTS_PD_U: k_xu_to_aos<<<nb, 256, 0, st>>>(s.xu[s.cur], dev_out, s.N, s.dim); break;
      case MTS_PD_V: k_soa_to_aos<<<nb, 256, 0, st>>>(s.v, dev_out, s.N, s.dim); break;
      case MTS_PD_A: k_soa_to_aos<<<nb, 256, 0, st>>>(s.a, dev_out, s.N, s.dim); break;
      case MTS_CONSTRAINT_NODES:
        k_index_to_double<<<(unsigned)((sz + 255) / 256), 256, 0, st>>>(s.cn, sz, dev_out);
        break;
      case MTS_FE_U: src = s.uF; break;
      case MTS_FE_V: src = s.vF; break;
      case MTS_FE_A: src = s.aF; break;
      case MTS_FE_X: src = s.xF; break;
      case MTS_FE_MASS: src = s.mF; break;
      case MTS_DAMAGE: pd_damage(s); src = s.damage; break;
      case MTS_PD_ALPHA: src = s.alpha; break;
      case MTS_PD_MASS: src = s.mass; break;
      case MTS_LAMBDA: src = s.lam0; break;
      case MTS_H: src = s.Hcopy; break;
      default: throw ArgError{"unknown quantity"};
    }
    MTS_LAUNCH_CHECK();
    if (src) MTS_HIP(hipMemcpyAsync(dev_out, src, sizeof(double) * sz, hipMemcpyDeviceToDevice, st));
    return MTS_OK;
  } catch (...) {
    return fail_from_exception();
  }
}

mts_status read_impl(Solver &s, int32_t what, double *out, int64_t cap, int64_t *n) {
  try {
    int64_t sz = qsize(s, what);
    if (sz < 0) throw ArgError{"quantity not available"};
    if (cap < sz) throw ArgError{"output capacity too small"};
    if (n) *n = sz;
    if (sz == 0) return MTS_OK;
    hipStream_t st = s.stream;
    const double *src = nullptr;
    double *tmp = nullptr;
    switch (what) {
      case MTS_PD_U: case MTS_PD_V: case MTS_PD_A: {
        tmp = s.arena.alloc<double>(sz);
        if (what == MTS_PD_U) {
          k_xu_to_aos<<<(unsigned)((s.N + 255) / 256), 256, 0, st>>>(s.xu[s.cur], tmp, s.N, s.dim);
        } else {
          const double *soa = what == MTS_PD_V ? s.v : s.a;
          k_soa_to_aos<<<(unsigned)((s.N + 255) / 256), 256, 0, st>>>(soa, tmp, s.N, s.dim);
        }
        MTS_LAUNCH_CHECK();
        src = tmp;
        break;
      }
      case MTS_FE_U: src = s.uF; break;
      case MTS_FE_V: src = s.vF; break;
      case MTS_FE_A: src = s.aF; break;
      case MTS_FE_X: src = s.xF; break;
      case MTS_FE_MASS: src = s.mF; break;
      case MTS_DAMAGE: pd_damage(s); src = s.damage; break;
      case MTS_PD_ALPHA: src = s.alpha; break;
      case MTS_PD_MASS: src = s.mass; break;
      case MTS_LAMBDA: src = s.lam0; break;
      case MTS_H: src = s.Hcopy; break;
      case MTS_CONSTRAINT_NODES:
        for (int64_t q = 0; q < s.nc; q++) out[q] = (double)s.h_cn[q];
        return MTS_OK;
      default: throw ArgError{"unknown quantity"};
    }
    MTS_HIP(hipMemcpyAsync(out, src, sizeof(double) * sz, hipMemcpyDeviceToHost, st));
    MTS_HIP(hipStreamSynchronize(st));
    if (tmp) s.arena.release(tmp);
    return MTS_OK;
  } catch (...) {
    return fail_from_exception();
  }
}
}  // namespace mts

extern "C" {

mts_status mts_write(mts_solver *h, int32_t what, const double *in, int64_t n) {
  if (!h || !in) return (std::snprintf(g_err, sizeof g_err, "null argument"), MTS_EINVAL);
  try {
    Solver &s = h->s;
    hipStream_t st = s.stream;
    if (what == MTS_PD_U || what == MTS_PD_V || what == MTS_PD_A) {
      if (n != s.N * s.dim) throw ArgError{"size mismatch"};
      double *tmp = s.arena.alloc<double>(n);
      MTS_HIP(hipMemcpyAsync(tmp, in, sizeof(double) * n, hipMemcpyHostToDevice, st));
      if (what == MTS_PD_U) {
        k_aos_to_xu<<<(unsigned)((s.N + 255) / 256), 256, 0, st>>>(tmp, s.xu[s.cur], s.N, s.dim);
      } else {
        double *dst = what == MTS_PD_V ? s.v : s.a;
        k_aos_to_soa<<<(unsigned)((s.N + 255) / 256), 256, 0, st>>>(tmp, dst, s.N, s.dim);
      }
      MTS_LAUNCH_CHECK();
      pd_predict_all(s);
      MTS_HIP(hipStreamSynchronize(st));
      s.arena.release(tmp);
      return MTS_OK;
    }
    double *dst = nullptr;
    int64_t want = 0;
    switch (what) {
      case MTS_FE_U: dst = s.uF; want = s.nfe * s.dim; break;
      case MTS_FE_V: dst = s.vF; want = s.nfe * s.dim; break;
      case MTS_FE_A: dst = s.aF; want = s.nfe * s.dim; break;
      case MTS_LAMBDA: dst = s.lam0; want = s.nl; break;
      default: throw ArgError{"quantity cannot be written"};
    }
    if (!dst || n != want) throw ArgError{"size mismatch or quantity not present"};
    MTS_HIP(hipMemcpyAsync(dst, in, sizeof(double) * n, hipMemcpyHostToDevice, st));
    MTS_HIP(hipStreamSynchronize(st));
    return MTS_OK;
  } catch (...) {
    return fail_from_exception();
  }
}

mts_status mts_read_bonds(mts_solver *h, int64_t *row_ptr, int32_t *col, uint8_t *intact, int64_t cap,
                          int64_t *nnz) {
  if (!h) return (std::snprintf(g_err, sizeof g_err, "null solver"), MTS_EINVAL);
  try {
    Solver &s = h->s;
    if (nnz) *nnz = s.nnz;
    if ((col || intact) && cap < s.nnz) throw ArgError{"capacity too small"};
    hipStream_t st = s.stream;
    if (row_ptr) {
      std::vector<int32_t> rp(s.N + 1);
      MTS_HIP(hipMemcpyAsync(rp.data(), s.rp, sizeof(int32_t) * (s.N + 1), hipMemcpyDeviceToHost, st));
      MTS_HIP(hipStreamSynchronize(st));
      for (int64_t i = 0; i <= s.N; i++) row_ptr[i] = rp[i];
    }
    if (col) MTS_HIP(hipMemcpyAsync(col, s.csr_col, sizeof(int32_t) * s.nnz, hipMemcpyDeviceToHost, st));
    if (intact) {
      uint8_t *tmp = s.arena.alloc<uint8_t>(s.nnz);
      bonds_to_csr_state(s, tmp);
      MTS_HIP(hipMemcpyAsync(intact, tmp, s.nnz, hipMemcpyDeviceToHost, st));
      MTS_HIP(hipStreamSynchronize(st));
      s.arena.release(tmp);
    }
    MTS_HIP(hipStreamSynchronize(st));
    return MTS_OK;
  } catch (...) {
    return fail_from_exception();
  }
}

mts_status mts_query(mts_solver *h, mts_info *o) {
  if (!h || !o) return (std::snprintf(g_err, sizeof g_err, "null argument"), MTS_EINVAL);
  query_impl(h->s, o);
  return MTS_OK;
}

}  // extern "C"

void mts::query_impl(Solver &s, mts_info *o) {
  std::memset(o, 0, sizeof *o);
  o->delta = s.prm.delta;
  o->volume = s.prm.V;
  o->c0 = s.prm.c0;
  o->s_crit = s.prm.scrit;
  o->dt_pd = s.prm.dtP;
  o->dt_fe = s.prm.dtF;
  o->n_pd = s.N;
  o->nnz = s.nnz;
  o->n_fe_nodes = s.nfe;
  o->n_fe_elems = s.ne;
  o->n_constraints = s.nc;
  o->n_region = s.n_region;
  o->pd_steps = s.pd_steps;
  o->macro_steps = s.macro_steps;
  o->n_rebuilds = s.n_rebuilds;
  o->n_rebuild_columns = s.n_rebuild_cols;
  o->n_colors = s.n_colors;
  o->device_bytes = (int64_t)s.arena.live;
  o->dim = s.dim;
  o->precision = s.precision;
  o->dt_bound_pd = s.dt_bound_pd;
  o->inverse_bytes = ((s.sym.kept ? s.sym.n_kept : s.sym.n_tiles) - s.sym.n_kept32) * 64 * 64 * (int64_t)sizeof(double) +
                     s.sym.n_kept32 * 64 * 64 * (int64_t)sizeof(float);
  o->slot_bytes = s.sell.pair_slots ? 6.0 : s.precision == MTS_MIXED ? 8.0 : 12.0;
}

extern "C" {

mts_status mts_profile(mts_solver *h, int32_t enable) {
  if (!h) return (std::snprintf(g_err, sizeof g_err, "null solver"), MTS_EINVAL);
  try {
    h->s.prof_collect();
    h->s.profiling = enable != 0;
    for (int k = 0; k < MTS_KT_COUNT; k++) {
      h->s.kt_ms[k] = 0.0;
      h->s.kt_count[k] = 0;
    }
    return MTS_OK;
  } catch (...) {
    return fail_from_exception();
  }
}

mts_status mts_kernel_time(mts_solver *h, int32_t kernel, int64_t *launches, double *total_ms) {
  if (!h || kernel < 0 || kernel >= MTS_KT_COUNT) return (std::snprintf(g_err, sizeof g_err, "bad argument"), MTS_EINVAL);
  try {
    h->s.prof_collect();
    if (launches) *launches = h->s.kt_count[kernel];
    if (total_ms) *total_ms = h->s.kt_ms[kernel];
    return MTS_OK;
  } catch (...) {
    return fail_from_exception();
  }
}

void mts_destroy(mts_solver *h) {
  if (!h) return;
  Solver &s = h->s;
  (void)hipStreamSynchronize(s.stream);
  for (int k = 0; k < MTS_KT_COUNT; k++)
    for (auto &pr : s.ev_pending[k]) {
      (void)hipEventDestroy(pr.e0);
      (void)hipEventDestroy(pr.e1);
    }
  for (hipEvent_t e : s.ev_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : s.flag_event)
    if (e) (void)hipEventDestroy(e);
  if (s.nf_event) (void)hipEventDestroy(s.nf_event);
  if (s.pinned_flag) (void)hipHostFree(s.pinned_flag);
  coupling_free(s);
  fe_implicit_free(s);
  pd_implicit_free(s);
  s.arena.free_all();
  delete h;
}

}  // extern "C"
