// Peridynamic subdomain on the device: Arlequin weights and masses, the fused
// substep kernel (bond stretch, irreversible breaking, pairwise force, velocity
// Verlet corrector and the next predictor), the link-problem substep used for
// the unit-load responses and for the final update, and nodal damage.
//
// Equations: Eq. 2 (force), Eq. 3 (stretch), Eq. 4 (bond state), Eq. 5 (damage),
// Eq. 38 with gamma = 1/2, beta = 0 (velocity Verlet), Eq. 48a/48b (free and
// link problems), Eq. 17-18 and Eq. 34 (Arlequin weights of stiffness and mass).
#include <cstdio>
#include <cstring>
#include <type_traits>

#include "device_math.h"
#include "fe_device.h"

namespace mts {

namespace {

constexpr int kBlock = 256;  // 4 wavefronts = 4 slices per workgroup

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

// predicted displacement (u part of the next node records)
__global__ void k_predict(int64_t N, int dim, double dt, double hdt2, const double *xu, const double *v,
                          const double *a, double *xu_next) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  for (int d = 0; d < dim; d++) {
    int64_t t = d * N + i, q = i * 2 * dim + dim + d;
    xu_next[q] = (xu[q] + dt * v[t]) + hdt2 * a[t];
  }
}

struct SubstepArgs {
  const double *x;
  const int32_t *rows;  // row -> node (rows in spatial tile order)
  int64_t N, n_slices;
  int T;
  const int32_t *width;
  const int64_t *slot_off, *word_off;
  const uint32_t *slots;  // per slot: record byte offset (LDS offset when staged) and coefficient;
                          // mixed staged pass: one record per two slots (see load_slot_chunk)
  const int32_t *halo_off, *halo_ids;  // per-workgroup staged neighbour lists (or nullptr)
  const int32_t *wg_start;             // staged pass: first slice of each workgroup
  uint64_t *mask;
  const double *mass, *P;
  const double *xu_in;  // node records [x, u_j (predicted)]
  double *xu_out;       // node records, u part <- u_{j+1} predicted
  double *v, *a;
  const int32_t *cidx;
  const double *lam0;
  double sfac;
  const uint8_t *in_region;
  int32_t *region_flag;
  int32_t *nonfinite;   // last substep: set when a new velocity is not finite
  const int32_t *rp;
  double *damage;       // written when non-null
  int breaking;
};

struct SubstepEntry {
  SubstepArgs A;
  Params P;
  int32_t first_block;
};

// One wavefront = one slice of 64/L consecutive nodes; the L lanes of a node
// take every L-th slot of its family, their partial sums are combined by a
// fixed butterfly (deterministic, no atomics).  Bond states of one iteration of
// the slice form one 64-bit word owned by the wavefront.
// Load through a uniform base pointer and a 32-bit byte offset (global loads
// with a scalar base: one address register per lane).  Offsets stay below 2^32
// for every array of a solver (checked when the layout is built).
template <class T>
__device__ __forceinline__ T ld32(const T *base, uint32_t byte_off) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}

// Raw slot data of TM consecutive iterations of a slice, as loaded (decoded
// only when the chunk runs).
template <int TM>
struct SlotChunk {
  uint64_t w[TM];           // bond-state words
  uint32_t c[TM];           // neighbour record byte offset (in LDS when staged)
  uint32_t f0[TM], f1[TM];  // coefficient bits (f1: high word, FP64 only)
};

// A zero the compiler cannot see through, in a vector register.  The state
// word of an iteration is the same in every lane; loading it through this
// lane-varying offset keeps it in vector registers, so a look-ahead load is not
// waited for at once to move it into scalar registers.
__device__ __forceinline__ uint32_t lane_zero() {
  uint32_t z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return z;
}

// Iterations t .. t + TM - 1 of the slice whose state words start at wo and
// whose slot index of (iteration 0, this lane) is so.
// PAIR (mixed form, staged pass): one record per two iterations,
// {coef(t), coef(t + 1), idx(t) | idx(t + 1) << 16} with idx the neighbour's
// position in the workgroup's LDS list; so is then the record index of
// (iterations 0 and 1, this lane) and t is even.  Both c entries of a pair
// keep the packed word, which is split where it is used.
template <bool MX, int TM, bool PAIR = false>
__device__ __forceinline__ void load_slot_chunk(const uint64_t *mask, const uint32_t *slots, int64_t wo, uint32_t so,
                                                uint32_t zoff, int t, SlotChunk<TM> &C) {
  if constexpr (PAIR) {
    static_assert(MX && TM % 2 == 0, "paired records: mixed form, whole pairs per chunk");
#pragma unroll
    for (int q = 0; q < TM; q++) C.w[q] = ld32(mask, (uint32_t)(wo + t + q) * 8u + zoff);
#pragma unroll
    for (int p = 0; p < TM / 2; p++) {
      const uint32_t rpos = so + (uint32_t)((t >> 1) + p) * WAVE;
      const uint3 v = ld32(reinterpret_cast<const uint3 *>(slots), rpos * 12u);
      C.f0[2 * p] = v.x;
      C.f0[2 * p + 1] = v.y;
      C.c[2 * p] = v.z;
      C.c[2 * p + 1] = v.z;
      C.f1[2 * p] = C.f1[2 * p + 1] = 0u;
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < TM; q++) {
    const uint32_t pos = so + (uint32_t)(t + q) * WAVE;
    C.w[q] = ld32(mask, (uint32_t)(wo + t + q) * 8u + zoff);
    if constexpr (MX) {
      const uint2 v = ld32(reinterpret_cast<const uint2 *>(slots), pos * 8u);  // {offset, coef}
      C.c[q] = v.x;
      C.f0[q] = v.y;
      C.f1[q] = 0u;
    } else {
      const uint3 v = ld32(reinterpret_cast<const uint3 *>(slots), pos * 12u);  // {coef lo, coef hi, offset}
      C.f0[q] = v.x;
      C.f1[q] = v.y;
      C.c[q] = v.z;
    }
  }
}

// A node record's 16-byte part, read either through the caches (ld32) or
// coherently with every chiplet's writes (COH: two agent-scope loads, which
// fetch from memory rather than from this chiplet's L2).
template <bool COH>
__device__ __forceinline__ double2 ld_rec(const double2 *base, uint32_t byte_off) {
  if constexpr (COH) {
    const uint64_t *p = reinterpret_cast<const uint64_t *>(reinterpret_cast<const char *>(base) + byte_off);
    const uint64_t a = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t b = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_double2(__longlong_as_double((long long)a), __longlong_as_double((long long)b));
  } else {
    return ld32(base, byte_off);
  }
}

template <int DIM, int L, bool MX, int TM, bool HALO = false, bool PAIR = false, bool COH = false>
__device__ __forceinline__ void substep_body(const SubstepArgs &A, const Params &P, const int64_t slice,
                                             const double2 *lds = nullptr, const SlotChunk<TM> *first = nullptr) {
  // MX: mixed form -- stretch, force and accumulation in FP32 on differences
  // formed in FP64; the accumulated value is the acceleration (coefficient
  // pre-divided by the node mass).  Integration stays FP64.
  using R = typename std::conditional<MX, float, double>::type;
  constexpr int S = WAVE / L;
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t N = A.N;
  const uint32_t N8 = (uint32_t)N * 8u;  // byte stride of one component
  const int jl = lane / L, l = lane % L;
  const int T = A.T;
  const int64_t wo = slice * T;
  // slot index of (iteration 0, this lane); with paired records, record index of (iterations 0 and 1)
  const uint32_t so = (uint32_t)((PAIR ? slice * ((T + 1) >> 1) : wo) * WAVE) + (uint32_t)lane;
  const uint32_t zoff = lane_zero();
  // The first chunk of slot data does not depend on the row's node: a caller
  // may have requested it already (before its staging loads).
  SlotChunk<TM> C0, C1;
  if (first) C0 = *first;
  const int64_t row = slice * S + jl;
  const bool valid = row < N;
  const int64_t i = valid ? A.rows[row] : 0;
  const uint32_t i8 = (uint32_t)i * 8u;
  constexpr uint32_t RB = 16u * DIM;  // bytes of one node record
  double xi_[DIM], ui_[DIM];
  {
    double rec[2 * DIM];
#pragma unroll
    for (int h = 0; h < DIM; h++) {
      const double2 v2 = ld_rec<COH>(reinterpret_cast<const double2 *>(A.xu_in), (uint32_t)i * RB + 16u * h);
      rec[2 * h] = v2.x;
      rec[2 * h + 1] = v2.y;
    }
#pragma unroll
    for (int d = 0; d < DIM; d++) {
      xi_[d] = rec[d];
      ui_[d] = rec[DIM + d];
    }
  }
  // node data of the corrector, fetched up front so it shares the first round trip
  double v_o[DIM], a_o[DIM], p_o[DIM];
  for (int d = 0; d < DIM; d++) {
    v_o[d] = ld32(A.v, i8 + d * N8);
    a_o[d] = ld32(A.a, i8 + d * N8);
    p_o[d] = A.P ? ld32(A.P, i8 + d * N8) : 0.0;
  }
  const int32_t q_i = A.cidx ? ld32(A.cidx, (uint32_t)i * 4u) : -1;
  const double m_i = ld32(A.mass, i8);
  R F[DIM];
  for (int d = 0; d < DIM; d++) F[d] = R(0);
  int n_intact = 0;
  int broke = 0;
  // Chunks of TM iterations, software-pipelined over two register sets: the
  // state words and slot records of chunk t + TM are requested before chunk t
  // is gathered and evaluated, and are only decoded when their own chunk runs,
  // so their memory latency overlaps a whole chunk of work.  The slot arrays
  // carry kSpareIters (>= 2 TM - 1) spare iterations past the last slice, so
  // every such load is in bounds; slots past T are masked out.
  static_assert(kSpareIters >= 2 * TM - 1, "spare iterations must cover the look-ahead chunk");
  const uint64_t lanebit = 1ull << lane;
  auto run_chunk = [&](int t0, const SlotChunk<TM> &C) {
    double xk[TM][DIM], uk[TM][DIM];
#pragma unroll
    for (int q = 0; q < TM; q++) {
      double rec[2 * DIM];
#pragma unroll
      for (int h = 0; h < DIM; h++) {
        double2 v2;
        if constexpr (PAIR) {
          const uint32_t idx = (q & 1) ? (C.c[q] >> 16) : (C.c[q] & 0xffffu);
          v2 = lds[idx * DIM + h];
        } else if constexpr (HALO) v2 = *reinterpret_cast<const double2 *>(reinterpret_cast<const char *>(lds) + C.c[q] + 16u * h);
        else v2 = ld32(reinterpret_cast<const double2 *>(A.xu_in), C.c[q] + 16u * h);
        rec[2 * h] = v2.x;
        rec[2 * h + 1] = v2.y;
      }
#pragma unroll
      for (int d = 0; d < DIM; d++) {
        xk[q][d] = rec[d];
        uk[q][d] = rec[DIM + d];
      }
    }
#pragma unroll
    for (int q = 0; q < TM; q++) {
      if (t0 + q >= T) break;  // wave-uniform: the rest of the chunk lies past the slice
      const uint64_t word = C.w[q];
      bool bit = (word & lanebit) != 0ull;
      bool cut = false;  // this lane's bond broke in this iteration
      if (bit) {
        if constexpr (!MX) {
          const R cf = __longlong_as_double((long long)(((uint64_t)C.f1[q] << 32) | C.f0[q]));
          double xi[DIM], eta[DIM];
          for (int d = 0; d < DIM; d++) {
            xi[d] = xk[q][d] - xi_[d];
            eta[d] = uk[q][d] - ui_[d];
          }
          if (A.breaking) {
            // squared lengths as the plain formula forms them (no contraction)
            double r2 = xi[0] * xi[0] + xi[1] * xi[1];
            double y0 = xi[0] + eta[0], y1 = xi[1] + eta[1];
            double y2 = y0 * y0 + y1 * y1;
            if (DIM == 3) {
              double yz = xi[2] + eta[2];
              r2 = r2 + xi[2] * xi[2];
              y2 = y2 + yz * yz;
            }
            if (breaks(r2, y2, P.K2, P.scrit)) {  // Eq. 3-4
              bit = false;
              broke = 1;
              cut = true;
            }
          }
          if (bit) {
            double xe = __builtin_fma(xi[1], eta[1], xi[0] * eta[0]);
            if (DIM == 3) xe = __builtin_fma(xi[2], eta[2], xe);
            const double tt = cf * xe;  // Eq. 2 times V_i V_k, Arlequin-weighted
            for (int d = 0; d < DIM; d++) F[d] = __builtin_fma(tt, xi[d], F[d]);
            n_intact++;
          }
        } else {
          const R cf = __uint_as_float(C.f0[q]);
          float xi[DIM], eta[DIM];
          for (int d = 0; d < DIM; d++) {
            xi[d] = (float)(xk[q][d] - xi_[d]);
            eta[d] = (float)(uk[q][d] - ui_[d]);
          }
          float xe = __builtin_fmaf(xi[1], eta[1], xi[0] * eta[0]);
          if (DIM == 3) xe = __builtin_fmaf(xi[2], eta[2], xe);
          if (A.breaking) {
            // |xi+eta|^2 - |xi|^2 = 2 xi.eta + eta.eta >= ((1+s_c)^2 - 1) |xi|^2
            float r2 = __builtin_fmaf(xi[1], xi[1], xi[0] * xi[0]);
            float ee = __builtin_fmaf(eta[1], eta[1], eta[0] * eta[0]);
            if (DIM == 3) {
              r2 = __builtin_fmaf(xi[2], xi[2], r2);
              ee = __builtin_fmaf(eta[2], eta[2], ee);
            }
            if (__builtin_fmaf(2.0f, xe, ee) >= P.K2m1f * r2) {
              bit = false;
              broke = 1;
              cut = true;
            }
          }
          if (bit) {
            const float tt = cf * xe;
            for (int d = 0; d < DIM; d++) F[d] = __builtin_fmaf(tt, xi[d], F[d]);
            n_intact++;
          }
        }
      }
      // bits only ever clear, so the word changes exactly when a lane cut a bond
      if (__any(cut)) {
        const uint64_t nw = __ballot(bit);
        if (lane == 0) A.mask[wo + t0 + q] = nw;
      }
    }
  };
  if (!first) load_slot_chunk<MX, TM, PAIR>(A.mask, A.slots, wo, so, zoff, 0, C0);
  for (int t0 = 0; t0 < T; t0 += 2 * TM) {
    load_slot_chunk<MX, TM, PAIR>(A.mask, A.slots, wo, so, zoff, t0 + TM, C1);
    run_chunk(t0, C0);
    if (t0 + TM >= T) break;
    load_slot_chunk<MX, TM, PAIR>(A.mask, A.slots, wo, so, zoff, t0 + 2 * TM, C0);
    run_chunk(t0 + TM, C1);
  }
  for (int off = L / 2; off >= 1; off >>= 1) {
    for (int d = 0; d < DIM; d++) F[d] += __shfl_xor(F[d], off, WAVE);
    n_intact += __shfl_xor(n_intact, off, WAVE);
    broke |= __shfl_xor(broke, off, WAVE);
  }
  if (!valid) return;
  if (l == 0 && broke && A.in_region && A.in_region[i]) A.region_flag[0] = 1;
  for (int d = 0; d < DIM; d++) {
    if (d % L != l) continue;
    const int64_t tix = d * N + i;
    double an;
    if constexpr (MX) {
      // F already holds the bond acceleration; external and multiplier forces in FP64
      double ext = p_o[d];
      if (q_i >= 0) ext = ext + A.sfac * A.lam0[q_i * DIM + d];
      an = (double)F[d] + ext / m_i;
    } else {
      double fl = F[d] + p_o[d];
      if (q_i >= 0) fl = fl + A.sfac * A.lam0[q_i * DIM + d];  // + G_P^T S_j
      an = fl / m_i;
    }
    const double vn = v_o[d] + P.hdtP * (a_o[d] + an);
    A.a[tix] = an;
    A.v[tix] = vn;
    if (A.nonfinite && !__builtin_isfinite(vn)) A.nonfinite[0] = 1;
    const double un = (ui_[d] + P.dtP * vn) + P.hdt2P * an;
    if constexpr (COH)  // written through to memory, where the other chiplets read it
      __hip_atomic_store(reinterpret_cast<uint64_t *>(A.xu_out + (int64_t)i * 2 * DIM + DIM + d),
                         (uint64_t)__double_as_longlong(un), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      A.xu_out[(int64_t)i * 2 * DIM + DIM + d] = un;
  }
  if (A.damage && l == 0) {
    const int fam = A.rp[i + 1] - A.rp[i];
    A.damage[i] = fam > 0 ? 1.0 - (double)n_intact / (double)fam : 0.0;
  }
}

// One solver: slice = renumbered workgroup * 4 + wavefront (wave-uniform, so
// offsets and state words come through scalar loads).
template <int DIM, int L, bool MX, int TM>
__global__ __launch_bounds__(kBlock) void k_pd_substep(SubstepArgs A, Params P) {
  const int64_t slice = __builtin_amdgcn_readfirstlane(
      (int)(xcd_block(blockIdx.x, gridDim.x) * (kBlock / WAVE) + (threadIdx.x >> 6)));
  if (slice >= A.n_slices) return;  // uniform per wavefront
  substep_body<DIM, L, MX, TM>(A, P, slice);
}

// Copy workgroup wg's neighbour records into LDS (all NT threads; a barrier follows).
template <int DIM, int NT, bool COH = false>
__device__ __forceinline__ void stage_halo(const SubstepArgs &A, int64_t wg, double2 *lds) {
  const int h0 = A.halo_off[wg], nh = A.halo_off[wg + 1] - h0;
  const double2 *src = reinterpret_cast<const double2 *>(A.xu_in);
  for (int h = threadIdx.x; h < nh; h += NT) {
    const uint32_t rb = (uint32_t)A.halo_ids[h0 + h] * (16u * DIM);
#pragma unroll
    for (int q = 0; q < DIM; q++) lds[h * DIM + q] = ld_rec<COH>(src, rb + 16u * q);
  }
}

// One solver, neighbour records staged in LDS per workgroup of up to NW
// wavefronts (consecutive slices of one spatial tile).  With NW = 8 the
// register budget is held to four wavefronts per SIMD, so that two workgroups
// share a CU.
template <int DIM, int L, bool MX, int NW, bool EARLY = (DIM == 2 && MX)>
__global__ __launch_bounds__(NW * 64, NW == 8 ? 4 : 1) void k_pd_substep_halo(SubstepArgs A, Params P) {
  extern __shared__ double2 lds[];
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int s0 = A.wg_start[b], w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const bool active = w < A.wg_start[b + 1] - s0;  // wave-uniform
  const int64_t slice = s0 + w;
  // the mixed form's staged pass reads paired slot records
  if constexpr (EARLY) {
    // the first chunk of slot data is requested before the staging loads
    SlotChunk<4> C0;
    if (active)
      load_slot_chunk<MX, 4, MX>(
          A.mask, A.slots, slice * A.T,
          (uint32_t)(slice * (MX ? (A.T + 1) >> 1 : A.T) * WAVE) + (threadIdx.x & (WAVE - 1)), lane_zero(), 0, C0);
    stage_halo<DIM, NW * 64>(A, b, lds);
    __syncthreads();
    if (!active) return;  // after the barrier every wave of the group has staged
    substep_body<DIM, L, MX, 4, true, MX>(A, P, slice, lds, &C0);
  } else {
    stage_halo<DIM, NW * 64>(A, b, lds);
    __syncthreads();
    if (!active) return;
    substep_body<DIM, L, MX, 4, true, MX>(A, P, slice, lds);
  }
}

// ---- the m substeps of a macro step in one launch (opt-in) ----
//
// Every workgroup of the staged pass stays resident for all m substeps of the
// free problem and keeps its tile.  Substep j of tile w needs the predicted
// displacements of substep j - 1 of every node its staged list holds, and it
// overwrites (in the other record buffer) the rows that other tiles staged in
// substep j - 1; both are covered by waiting until every tile in w's
// dependency list (a symmetric relation, built with the layout) has finished
// substep j - 1.  The node records are written and read coherently across the
// chiplets (agent-scope accesses, which go to memory rather than to a
// chiplet's own L2), so no cache-wide write-back or invalidation is needed:
// each wavefront waits for its stores to complete, then one thread publishes
// "finished substep j" as base + j in the tile's flag; a waiting tile polls
// its dependencies' flags.  Every wait is bounded: after spin_limit polls it
// sets the give-up flag and goes on, so the kernel always ends (the host then
// reports the solve as failed).  The launch is cooperative, so every
// workgroup is resident.
struct SubcycleArgs {
  SubstepArgs A;              // substep 1 (xu_in, xu_out swap every substep)
  double *damage;             // written by substep m
  int32_t *nonfinite;         // [0] non-finite velocity (substep m), [1] a wait gave up
  const int32_t *dep_off, *dep_ids;
  uint32_t *flags;            // per workgroup
  uint32_t base;              // flag value after substep j: base + j
  uint32_t spin_limit;
  int m;
};

// Publish "this workgroup finished substep value - base" once every
// wavefront's coherent record stores have completed.
__device__ __forceinline__ void subcycle_publish(const SubcycleArgs &S, int b, uint32_t value) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(S.flags + b, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until every dependency of workgroup b published at least `target`
// (lanes of the first wavefront poll one dependency each).
__device__ __forceinline__ void subcycle_wait(const SubcycleArgs &S, int b, uint32_t target) {
  if (threadIdx.x < WAVE) {
    const int d0 = S.dep_off[b], nd = S.dep_off[b + 1] - d0;
    for (int k = (int)threadIdx.x; k < nd; k += WAVE) {
      const uint32_t *f = S.flags + S.dep_ids[d0 + k];
      uint32_t polls = 0;
      while ((int32_t)(__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
        if (++polls > S.spin_limit ||
            __hip_atomic_load(S.nonfinite + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          __hip_atomic_store(S.nonfinite + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
  }
  __syncthreads();
}

template <int DIM, int L, bool MX, int NW>
__global__ __launch_bounds__(NW * 64, NW == 8 ? 4 : 1) void k_pd_subcycle_halo(SubcycleArgs S, Params P) {
  extern __shared__ double2 lds[];
  const int b = xcd_block(blockIdx.x, gridDim.x);
  SubstepArgs A = S.A;
  const int s0 = A.wg_start[b], w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const bool active = w < A.wg_start[b + 1] - s0;  // wave-uniform
  const int64_t slice = s0 + w;
  double *const buf0 = const_cast<double *>(A.xu_in), *const buf1 = A.xu_out;
  for (int j = 1; j <= S.m; j++) {
    A.xu_in = (j & 1) ? buf0 : buf1;
    A.xu_out = (j & 1) ? buf1 : buf0;
    A.sfac = 1.0 - (double)j / (double)S.m;
    A.damage = j == S.m ? S.damage : nullptr;
    A.nonfinite = j == S.m ? S.nonfinite : nullptr;
    if (j > 1) subcycle_wait(S, b, S.base + (uint32_t)(j - 1));
    stage_halo<DIM, NW * 64, true>(A, b, lds);
    __syncthreads();
    if (active) substep_body<DIM, L, MX, 4, true, MX, true>(A, P, slice, lds);
    subcycle_publish(S, b, S.base + (uint32_t)j);
  }
}

// Several solvers in one launch: workgroup b (after renumbering) belongs to
// solver blk_req[b], whose slices start at its entry's first_block.
template <int DIM, int L, bool MX>
__global__ __launch_bounds__(kBlock) void k_pd_substep_batch(const SubstepEntry *tab, const int32_t *blk_req) {
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int r = __builtin_amdgcn_readfirstlane(blk_req[b]);
  const SubstepArgs A = tab[r].A;
  const Params P = tab[r].P;
  const int64_t slice = __builtin_amdgcn_readfirstlane(
      (int)((b - tab[r].first_block) * (kBlock / WAVE) + (threadIdx.x >> 6)));
  if (slice >= A.n_slices) return;
  substep_body<DIM, L, MX, 4>(A, P, slice);
}

// Link problem (Eq. 48b / eq. unit): linear, no breaking, bond states of the
// last rebuild, the response starting from rest at substep 1.
//
// Unit-load responses (setup and rebuild): NRHS right-hand sides share one pass
// over the bond data; RHS b loads (j/m) e_dir(b) at every constraint node of
// colour(b).  The responses are node-major, [N][NRHS][DIM], so a neighbour's
// NRHS x DIM values are one contiguous run of 16-byte loads.
struct LinkArgs {
  const double *xrec;     // node records [x, u] of the free problem (x part read)
  int64_t N, n_rows, n_slices;
  int T;
  const int32_t *rows, *slice_layer;
  int jmax;               // rows farther than jmax horizons still hold exact zeros
  const int32_t *col;
  const double *coef;
  const uint64_t *mask;
  const double *mass;
  const double *u_in;
  double *u_out, *v, *a;  // [N][NRHS][DIM]
  const int32_t *cidx;
  const int32_t *ccolor;  // colour of each constraint
  int32_t rhs_color[16];
  int32_t rhs_dir[16];
  double lfac;
  int first;              // substep 1: the response starts from rest (inputs are exact zeros)
};

template <int DIM, int NRHS, int L>
__device__ __forceinline__ void link_body(const LinkArgs &A, const Params &P, const int64_t slice) {
  constexpr int S = WAVE / L, C = NRHS * DIM;  // C: values per node (even)
  static_assert(C % 2 == 0, "responses are loaded in pairs");
  const int lane = threadIdx.x & (WAVE - 1);
  const int jl = lane / L, l = lane % L;
  const int64_t r = slice * S + jl;
  const bool valid = r < A.n_rows;
  const int64_t i = valid ? A.rows[r] : A.rows[0];
  if (A.slice_layer[slice] > A.jmax) {  // uniform per wavefront
    // the response has not reached these rows yet: it is exactly zero
    if (!valid) return;
    for (int e = l; e < C; e += L) {
      A.u_out[i * C + e] = 0.0;
      if (A.first) {
        A.v[i * C + e] = 0.0;
        A.a[i * C + e] = 0.0;
      }
    }
    return;
  }
  const int T = A.T;
  const int64_t wo = slice * T, so = wo * WAVE;
  double xi_[DIM], ui_[C];
  for (int d = 0; d < DIM; d++) xi_[d] = A.xrec[i * 2 * DIM + d];
  {
    const double2 *src = reinterpret_cast<const double2 *>(A.u_in + i * C);
#pragma unroll
    for (int e = 0; e < C / 2; e++) {
      const double2 v2 = A.first ? double2{0.0, 0.0} : src[e];
      ui_[2 * e] = v2.x;
      ui_[2 * e + 1] = v2.y;
    }
  }
  double F[C];
#pragma unroll
  for (int e = 0; e < C; e++) F[e] = 0.0;
  for (int t = 0; t < (A.first ? 0 : T); t++) {  // no bond forces from a response at rest
    const int64_t pos = so + (int64_t)t * WAVE + lane;
    if (!((A.mask[wo + t] >> lane) & 1ull)) continue;
    const int64_t c = A.col[pos];
    const double cf = A.coef[pos];
    double xk[DIM], uk[C];
    for (int d = 0; d < DIM; d++) xk[d] = A.xrec[c * 2 * DIM + d];
    const double2 *src = reinterpret_cast<const double2 *>(A.u_in + c * C);
#pragma unroll
    for (int e = 0; e < C / 2; e++) {
      const double2 v2 = src[e];
      uk[2 * e] = v2.x;
      uk[2 * e + 1] = v2.y;
    }
    double xi[DIM];
    for (int d = 0; d < DIM; d++) xi[d] = xk[d] - xi_[d];
#pragma unroll
    for (int b = 0; b < NRHS; b++) {
      double xe = xi[0] * (uk[b * DIM] - ui_[b * DIM]) + xi[1] * (uk[b * DIM + 1] - ui_[b * DIM + 1]);
      if (DIM == 3) xe = xe + xi[2] * (uk[b * DIM + 2] - ui_[b * DIM + 2]);
      const double tt = cf * xe;
      for (int d = 0; d < DIM; d++) F[b * DIM + d] += tt * xi[d];
    }
  }
  for (int off = L / 2; off >= 1; off >>= 1)
#pragma unroll
    for (int e = 0; e < C; e++) F[e] += __shfl_xor(F[e], off, WAVE);
  if (!valid) return;
  const int32_t q = A.cidx[i];
  const double m_i = A.mass[i];
  const int32_t qc = q >= 0 ? A.ccolor[q] : -1;
#pragma unroll
  for (int e = 0; e < C; e++) {
    if (e % L != l) continue;
    const int b = e / DIM, d = e % DIM;
    const int64_t tix = i * C + e;
    double fl = F[e];
    if (qc >= 0 && qc == A.rhs_color[b] && d == A.rhs_dir[b]) fl = fl + A.lfac;
    const double an = fl / m_i;
    const double v0 = A.first ? 0.0 : A.v[tix], a0 = A.first ? 0.0 : A.a[tix];
    const double vn = v0 + P.hdtP * (a0 + an);
    A.a[tix] = an;
    A.v[tix] = vn;
    A.u_out[tix] = (ui_[e] + P.dtP * vn) + P.hdt2P * an;
  }
}

template <int DIM, int NRHS, int L>
__global__ __launch_bounds__(kBlock) void k_link_substep(LinkArgs A, Params P) {
  const int64_t slice = __builtin_amdgcn_readfirstlane(
      (int)(xcd_block(blockIdx.x, gridDim.x) * (kBlock / WAVE) + (threadIdx.x >> 6)));
  if (slice >= A.n_slices) return;
  link_body<DIM, NRHS, L>(A, P, slice);
}

// Final update of a macro step (Eq. 50): one right-hand side, the load
// (j/m) lambda_m at every constraint node.  The response lives in node records
// [x, w] (double-buffered like the free problem's) and the pass has the free
// problem's shape: interleaved slot records {coefficient, record offset},
// one 16-byte load per record half, chunks software-pipelined over two
// register sets.  At the last substep the response is added into the PD state.
struct Link1Args {
  int64_t N, n_rows, n_slices;
  int T;
  const int32_t *rows, *slice_layer;
  int jmax;               // rows farther than jmax horizons still hold exact zeros
  const uint32_t *slots;  // per slot: {coef lo, coef hi, record byte offset}
  const uint64_t *mask;
  const double *mass;
  const double *w_in;     // records [x, w_j]
  double *w_out;          // records, w part <- w_{j+1}
  double *v, *a;          // [DIM][N]
  const int32_t *cidx;
  const double *lam;
  double lfac;
  int first;              // substep 1: the response starts from rest
  // last substep: add W_m into the PD state (its displacement is this
  // substep's input) and write the next predictor, instead of storing W_m
  int add;
  double *Uxu, *Uxu_pred, *Uv, *Ua;
  // staged form: workgroup b runs slices wg_start[b] .. wg_start[b + 1] - 1
  // and first copies the records halo_ids[halo_off[b] ..] into LDS
  const int32_t *wg_start, *halo_off, *halo_ids;
  // workgroups past n_link_blocks run an independent FE pass (side): the FE
  // ring correction, or the next macro step's element forces or gather
  int64_t n_link_blocks;
  int side;
  FeRingArgs ring;
  FeElemArgs elem;
  FeGatherArgs gather;
  // kSideSnap: copy the free problem's bond states, then clear the rebuild flag
  const uint64_t *snap_src;
  uint64_t *snap_dst;
  int64_t snap_n;
  int32_t *snap_flag;
};

// (the Hex8 element pass would raise the 3D link kernel's register count, so
// the next FE free step joins the link launches in 2D only)
template <int DIM>
__device__ __forceinline__ void link_side_pass(const Link1Args &A, int64_t bb) {
  const int64_t g = bb * kBlock + threadIdx.x;
  if (A.side == kSideRing) fe_correct_ring_wave(A.ring, g / WAVE, (int)(threadIdx.x & (WAVE - 1)));
  if (A.side == kSideSnap) {
    if (g < A.snap_n) A.snap_dst[g] = A.snap_src[g];
    if (g == 0) A.snap_flag[0] = 0;
  }
  if constexpr (DIM == 2) {
    if (A.side == kSideElem) fe_elem_force_one<DIM, true>(A.elem, g);
    else if (A.side == kSideGather) fe_gather_free_one(A.gather, g);
  }
}

template <int DIM, int L, bool HALO>
__global__ __launch_bounds__(kBlock) void k_link_final(Link1Args A, Params P) {
  constexpr int S = WAVE / L, TM = 4;
  constexpr uint32_t RB = 16u * DIM;
  static_assert(kSpareIters >= 2 * TM - 1, "spare iterations must cover the look-ahead chunk");
  extern __shared__ double2 lds[];
  if ((int64_t)blockIdx.x >= A.n_link_blocks) {  // uniform per workgroup
    link_side_pass<DIM>(A, (int64_t)blockIdx.x - A.n_link_blocks);
    return;
  }
  const int nlb = (int)A.n_link_blocks;
  int64_t slice;
  if constexpr (HALO) {
    const int b = xcd_block(blockIdx.x, nlb);
    if (!A.first) {  // the first substep has no bond loop: nothing to stage (uniform per launch)
      const int h0 = A.halo_off[b], nh = A.halo_off[b + 1] - h0;
      const double2 *src = reinterpret_cast<const double2 *>(A.w_in);
      for (int h = threadIdx.x; h < nh; h += kBlock) {
        const uint32_t rb = (uint32_t)A.halo_ids[h0 + h] * RB;
#pragma unroll
        for (int q = 0; q < DIM; q++) lds[h * DIM + q] = ld32(src, rb + 16u * q);
      }
      __syncthreads();
    }
    const int s0 = A.wg_start[b], w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (w >= A.wg_start[b + 1] - s0) return;  // after the barrier every wave of the group has staged
    slice = s0 + w;
  } else {
    slice = __builtin_amdgcn_readfirstlane((int)(xcd_block(blockIdx.x, nlb) * (kBlock / WAVE) + (threadIdx.x >> 6)));
    if (slice >= A.n_slices) return;
  }
  const int lane = threadIdx.x & (WAVE - 1);
  const int jl = lane / L, l = lane % L;
  const int64_t r = slice * S + jl;
  const bool valid = r < A.n_rows;
  const int64_t N = A.N;
  if (A.slice_layer[slice] > A.jmax) {  // uniform per wavefront: not reached yet, exactly zero
    if (!valid) return;
    const int64_t i = A.rows[r];
    for (int d = l; d < DIM; d += L) {
      A.w_out[i * 2 * DIM + DIM + d] = 0.0;
      if (A.first) {
        A.v[d * N + i] = 0.0;
        A.a[d * N + i] = 0.0;
      }
    }
    return;
  }
  const int T = A.T;
  const int64_t wo = slice * T;
  const uint32_t so = (uint32_t)(wo * WAVE) + (uint32_t)lane;
  const uint32_t zoff = lane_zero();
  SlotChunk<TM> C0, C1;  // the first chunk is requested before the row's node data
  if (!A.first) load_slot_chunk<false, TM>(A.mask, A.slots, wo, so, zoff, 0, C0);
  const int64_t i = valid ? A.rows[r] : A.rows[0];
  double xi_[DIM], wi_[DIM];
  {
    double rec[2 * DIM];
#pragma unroll
    for (int h = 0; h < DIM; h++) {
      const double2 v2 = ld32(reinterpret_cast<const double2 *>(A.w_in), (uint32_t)i * RB + 16u * h);
      rec[2 * h] = v2.x;
      rec[2 * h + 1] = v2.y;
    }
#pragma unroll
    for (int d = 0; d < DIM; d++) {
      xi_[d] = rec[d];
      wi_[d] = A.first ? 0.0 : rec[DIM + d];
    }
  }
  // node data of the epilogue, requested before the bond loop
  const int32_t q = A.cidx[i];
  const double m_i = A.mass[i];
  double v0[DIM], a0[DIM], lq[DIM];
  for (int d = 0; d < DIM; d++) {
    v0[d] = A.first ? 0.0 : A.v[d * N + i];
    a0[d] = A.first ? 0.0 : A.a[d * N + i];
  }
  double F[DIM];
  for (int d = 0; d < DIM; d++) F[d] = 0.0;
  if (!A.first) {  // no bond forces from a response at rest
    const uint64_t lanebit = 1ull << lane;
    auto run_chunk = [&](int t0, const SlotChunk<TM> &C) {
      double xk[TM][DIM], wk[TM][DIM];
#pragma unroll
      for (int q = 0; q < TM; q++) {
        double rec[2 * DIM];
#pragma unroll
        for (int h = 0; h < DIM; h++) {
          double2 v2;
          if constexpr (HALO) v2 = *reinterpret_cast<const double2 *>(reinterpret_cast<const char *>(lds) + C.c[q] + 16u * h);
          else v2 = ld32(reinterpret_cast<const double2 *>(A.w_in), C.c[q] + 16u * h);
          rec[2 * h] = v2.x;
          rec[2 * h + 1] = v2.y;
        }
#pragma unroll
        for (int d = 0; d < DIM; d++) {
          xk[q][d] = rec[d];
          wk[q][d] = rec[DIM + d];
        }
      }
#pragma unroll
      for (int q = 0; q < TM; q++) {
        const uint64_t word = t0 + q < T ? C.w[q] : 0ull;
        if (word & lanebit) {
          const double cf = __longlong_as_double((long long)(((uint64_t)C.f1[q] << 32) | C.f0[q]));
          double xi[DIM];
          for (int d = 0; d < DIM; d++) xi[d] = xk[q][d] - xi_[d];
          double xe = __builtin_fma(xi[1], wk[q][1] - wi_[1], xi[0] * (wk[q][0] - wi_[0]));
          if (DIM == 3) xe = __builtin_fma(xi[2], wk[q][2] - wi_[2], xe);
          const double tt = cf * xe;
          for (int d = 0; d < DIM; d++) F[d] = __builtin_fma(tt, xi[d], F[d]);
        }
      }
    };
    for (int d = 0; d < DIM; d++) lq[d] = q >= 0 ? A.lam[q * DIM + d] : 0.0;  // in flight during the loop
    for (int t0 = 0; t0 < T; t0 += 2 * TM) {
      load_slot_chunk<false, TM>(A.mask, A.slots, wo, so, zoff, t0 + TM, C1);
      run_chunk(t0, C0);
      if (t0 + TM >= T) break;
      load_slot_chunk<false, TM>(A.mask, A.slots, wo, so, zoff, t0 + 2 * TM, C0);
      run_chunk(t0 + TM, C1);
    }
  }
  if (A.first)
    for (int d = 0; d < DIM; d++) lq[d] = q >= 0 ? A.lam[q * DIM + d] : 0.0;
  for (int off = L / 2; off >= 1; off >>= 1)
    for (int d = 0; d < DIM; d++) F[d] += __shfl_xor(F[d], off, WAVE);
  if (!valid) return;
  for (int d = l; d < DIM; d += L) {
    const int64_t t = d * N + i, qx = i * 2 * DIM + DIM + d;
    double fl = F[d];
    if (q >= 0) fl = fl + A.lfac * lq[d];
    const double an = fl / m_i;
    const double vn = v0[d] + P.hdtP * (a0[d] + an);
    if (A.add) {
      // U = V + W_m on this row, then the predictor for the next substep
      const double uu = A.Uxu[qx] + wi_[d];
      const double vv = A.Uv[t] + vn;
      const double aa = A.Ua[t] + an;
      A.Uxu[qx] = uu;
      A.Uv[t] = vv;
      A.Ua[t] = aa;
      A.Uxu_pred[qx] = (uu + P.dtP * vv) + P.hdt2P * aa;
    } else {
      A.a[t] = an;
      A.v[t] = vn;
      A.w_out[qx] = (wi_[d] + P.dtP * vn) + P.hdt2P * an;
    }
  }
}

// Node records [x, 0] of the final-update response.
__global__ void k_link_records(const double *x, int64_t N, int dim, double *rec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  for (int d = 0; d < dim; d++) {
    rec[i * 2 * dim + d] = x[d * N + i];
    rec[i * 2 * dim + dim + d] = 0.0;
  }
}

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// Stability bound of the explicit PD step at node i (the Silling-Askari
// criterion with the Arlequin bond weights): sqrt(2 m_i / sum_k w c |xi|^2 V_i V_k).
__global__ void k_pd_dt_bound(int64_t N, int dim, const double *x, const int32_t *rp, const int32_t *row_of, int L,
                              const int64_t *slot_off, const int32_t *col, const double *coef, const double *mass,
                              double *dt_node) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int64_t r = row_of ? row_of[i] : i;
  const int S = WAVE / L;
  double k = 0.0;
  for (int q = 0; q < rp[i + 1] - rp[i]; q++) {
    const int64_t pos = sell_slot(slot_off[r / S], (int)(r % S), q, L);
    const int64_t c = col[pos];
    double r2 = 0.0;
    for (int d = 0; d < dim; d++) {
      const double t = x[d * N + c] - x[d * N + i];
      r2 += t * t;
    }
    k += coef[pos] * r2;
  }
  dt_node[i] = k > 0.0 ? sqrt(2.0 * mass[i] / k) : 1e300;
}

// smallest of n values (one workgroup; the minimum does not depend on the order)
__global__ void k_min(const double *a, int64_t n, double *out) {
  __shared__ double part[256];
  double m = 1e300;
  for (int64_t i = threadIdx.x; i < n; i += 256) m = fmin(m, a[i]);
  part[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] = fmin(part[threadIdx.x], part[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0];
}

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
  sell_coefficients(s, s.sell);
  {
    // the step must respect the PD stability bound (an explicit step above it
    // grows without limit)
    double *t = s.arena.alloc<double>(N + 1);
    k_pd_dt_bound<<<nblk(N), 256, 0, st>>>(N, s.dim, s.x, s.rp, s.sell.row_of, s.sell.L, s.sell.slot_off,
                                           s.sell.col, s.sell.coef, s.mass, t);
    MTS_LAUNCH_CHECK();
    k_min<<<1, 256, 0, st>>>(t, N, t + N);
    MTS_LAUNCH_CHECK();
    double bound = 0.0;
    MTS_HIP(hipMemcpyAsync(&bound, t + N, sizeof(double), hipMemcpyDeviceToHost, st));
    MTS_HIP(hipStreamSynchronize(st));
    s.arena.release(t);
    s.dt_bound_pd = bound;
    if (s.prm.dtP > bound && !(s.pd_beta > 0.0)) {  // the implicit step has no such bound
      char msg[160];
      std::snprintf(msg, sizeof msg, "dt_pd = %.4g s exceeds the PD stability bound %.4g s", s.prm.dtP, bound);
      throw ArgError{msg};
    }
  }
  sell_pack_slots(s, s.sell);
  if (s.halo) sell_build_halo(s, s.sell);
}

void pd_predict_all(Solver &s) {
  k_predict<<<nblk(s.N), 256, 0, s.stream>>>(s.N, s.dim, s.prm.dtP, s.prm.hdt2P, s.xu[s.cur], s.v, s.a,
                                             s.xu[s.cur ^ 1]);
  MTS_LAUNCH_CHECK();
}

// Arguments of substep j (1..m) with displacement buffers u[cur ^ 1] (predicted
// u_j, read) and u[cur] (predicted u_{j+1}, written).
static SubstepArgs substep_args(Solver &s, int j, int cur) {
  SubstepArgs A{};
  A.x = s.x;
  A.rows = s.sell.rows;
  A.N = s.N;
  A.n_slices = s.sell.n_slices;
  A.T = s.sell.T;
  A.width = s.sell.width;
  A.slot_off = s.sell.slot_off;
  A.word_off = s.sell.word_off;
  A.slots = s.sell.slots;
  A.halo_off = s.sell.halo_max ? s.sell.halo_off : nullptr;
  A.halo_ids = s.sell.halo_max ? s.sell.halo_ids : nullptr;
  A.wg_start = s.sell.halo_max ? s.sell.wg_start : nullptr;
  A.mask = s.sell.mask;
  A.mass = s.mass;
  A.P = s.P;
  A.xu_in = s.xu[cur ^ 1];
  A.xu_out = s.xu[cur];
  A.v = s.v;
  A.a = s.a;
  A.cidx = s.nc ? s.cidx : nullptr;
  A.lam0 = s.lam0;
  A.sfac = 1.0 - (double)j / (double)s.m;
  A.in_region = s.nc ? s.in_region : nullptr;
  A.region_flag = s.region_flag;
  A.nonfinite = (j == s.m) ? s.nonfinite_flag : nullptr;
  A.rp = s.rp;
  A.damage = (j == s.m) ? s.damage : nullptr;
  A.breaking = s.breaking ? 1 : 0;
  return A;
}

#define MTS_BY_LANES(L, MACRO, D, MX)  \
  if (L == 1) MACRO(D, 1, MX);         \
  else if (L == 2) MACRO(D, 2, MX);    \
  else if (L == 4) MACRO(D, 4, MX);    \
  else MACRO(D, 8, MX)
#define MTS_BY_FORM(dim, mx, L, MACRO)                                   \
  if (dim == 2) {                                                        \
    if (mx) { MTS_BY_LANES(L, MACRO, 2, true); } else { MTS_BY_LANES(L, MACRO, 2, false); } \
  } else {                                                               \
    if (mx) { MTS_BY_LANES(L, MACRO, 3, true); } else { MTS_BY_LANES(L, MACRO, 3, false); } \
  }

// Substep j (1..m) of the free problem.  Reads u[cur^1] (predicted u_j), writes
// the predicted u_{j+1} into u[cur]; afterwards cur flips.
void pd_substep(Solver &s, int j) {
  const SubstepArgs A = substep_args(s, j, s.cur);
  const unsigned grid = (unsigned)((A.n_slices * WAVE + kBlock - 1) / kBlock);
  const int L = s.sell.L;
  if (s.sell.halo_max > 0) {
    // the staged pass reads paired slot records in the mixed form
    if ((s.precision == MTS_MIXED) != s.sell.pair_slots)
      throw ArgError{"internal: staged pass slot record layout mismatch"};
    const size_t shm = (size_t)s.sell.halo_max * 16 * s.dim;
    const int nw = s.sell.wg_waves;
    const unsigned hgrid = (unsigned)s.sell.n_wg;
    if (nw == 8) {
#define MTS_SUBH(D, LL, MX) k_pd_substep_halo<D, LL, MX, 8><<<hgrid, 8 * WAVE, shm, s.stream>>>(A, s.prm)
      MTS_BY_FORM(s.dim, s.precision == MTS_MIXED, L, MTS_SUBH);
#undef MTS_SUBH
    } else {
#define MTS_SUBH(D, LL, MX) k_pd_substep_halo<D, LL, MX, 4><<<hgrid, 4 * WAVE, shm, s.stream>>>(A, s.prm)
      MTS_BY_FORM(s.dim, s.precision == MTS_MIXED, L, MTS_SUBH);
#undef MTS_SUBH
    }
    MTS_LAUNCH_CHECK();
    s.cur ^= 1;
    s.pd_steps++;
    return;
  }
  switch (s.pd_variant) {  // chunk length (iterations per pipelined chunk)
#define MTS_SUB(D, LL, MX) k_pd_substep<D, LL, MX, 2><<<grid, kBlock, 0, s.stream>>>(A, s.prm)
    case 1: MTS_BY_FORM(s.dim, s.precision == MTS_MIXED, L, MTS_SUB); break;
#undef MTS_SUB
#define MTS_SUB(D, LL, MX) k_pd_substep<D, LL, MX, 8><<<grid, kBlock, 0, s.stream>>>(A, s.prm)
    case 2: MTS_BY_FORM(s.dim, s.precision == MTS_MIXED, L, MTS_SUB); break;
#undef MTS_SUB
#define MTS_SUB(D, LL, MX) k_pd_substep<D, LL, MX, 4><<<grid, kBlock, 0, s.stream>>>(A, s.prm)
    default: MTS_BY_FORM(s.dim, s.precision == MTS_MIXED, L, MTS_SUB); break;
#undef MTS_SUB
  }
  MTS_LAUNCH_CHECK();
  s.cur ^= 1;
  s.pd_steps++;
}

// All m substeps of the free problem as one launch of the staged pass, when
// every workgroup of it can be resident at once; reads u[cur ^ 1] like
// substep 1 and leaves cur flipped m times.
bool pd_subcycle(Solver &s) {
  if (!s.subcycle || s.sell.halo_max <= 0 || !s.sell.dep_off || s.m < 2) return false;
  if ((s.precision == MTS_MIXED) != s.sell.pair_slots) return false;
  const int L = s.sell.L;
  const int nw = s.sell.wg_waves;
  const size_t shm = (size_t)s.sell.halo_max * 16 * s.dim;
  const void *fn = nullptr;
#define MTS_SUBC(D, LL, MX)                                                                  \
  fn = nw == 8 ? reinterpret_cast<const void *>(&k_pd_subcycle_halo<D, LL, MX, 8>)          \
               : reinterpret_cast<const void *>(&k_pd_subcycle_halo<D, LL, MX, 4>)
  MTS_BY_FORM(s.dim, s.precision == MTS_MIXED, L, MTS_SUBC);
#undef MTS_SUBC
  if (s.sub_capacity < 0) {
    int per_cu = 0, n_cu = 0;
    MTS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, nw * 64, shm));
    MTS_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, s.device));
    s.sub_capacity = per_cu * n_cu;
  }
  if (s.sell.n_wg > s.sub_capacity) return false;
  SubcycleArgs S{};
  S.A = substep_args(s, 1, s.cur);
  S.damage = s.damage;
  S.nonfinite = s.nonfinite_flag;
  S.dep_off = s.sell.dep_off;
  S.dep_ids = s.sell.dep_ids;
  S.flags = s.sell.wg_flag;
  S.base = s.sub_epoch;
  S.spin_limit = s.spin_limit;
  S.m = s.m;
  void *args[] = {&S, &s.prm};
  MTS_HIP(hipLaunchCooperativeKernel(fn, dim3((unsigned)s.sell.n_wg), dim3((unsigned)(nw * 64)), args,
                                     (unsigned)shm, s.stream));
  s.sub_epoch += (uint32_t)s.m;
  if (s.m & 1) s.cur ^= 1;
  s.pd_steps += s.m;
  return true;
}

// ---- batched substeps over several solvers (serving pool) ----
size_t substep_entry_size() { return sizeof(SubstepEntry); }

int64_t substep_blocks(const Solver &s) { return (s.sell.n_slices * WAVE + kBlock - 1) / kBlock; }

void substep_entry_fill(Solver &s, int j, int cur, int32_t first_block, void *dst) {
  SubstepEntry e{};
  e.A = substep_args(s, j, cur);
  e.P = s.prm;
  e.first_block = first_block;
  std::memcpy(dst, &e, sizeof e);
}

void substep_batch_launch(int dim, bool mixed, int L, const void *dev_tab, const int32_t *dev_blk_req,
                          int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return;
  const SubstepEntry *tab = static_cast<const SubstepEntry *>(dev_tab);

#define MTS_SUBB(D, LL, MX) k_pd_substep_batch<D, LL, MX><<<(unsigned)nblocks, kBlock, 0, st>>>(tab, dev_blk_req)
  MTS_BY_FORM(dim, mixed, L, MTS_SUBB);
#undef MTS_SUBB
  MTS_LAUNCH_CHECK();
}

// ---- link runs (used by coupling.hip) ----

template <int DIM, int NRHS>
static void launch_link(Solver &s, LinkArgs &A) {
  unsigned grid = (unsigned)((A.n_slices * WAVE + kBlock - 1) / kBlock);
  switch (s.rsell.L) {
    case 1: k_link_substep<DIM, NRHS, 1><<<grid, kBlock, 0, s.stream>>>(A, s.prm); break;
    case 2: k_link_substep<DIM, NRHS, 2><<<grid, kBlock, 0, s.stream>>>(A, s.prm); break;
    case 4: k_link_substep<DIM, NRHS, 4><<<grid, kBlock, 0, s.stream>>>(A, s.prm); break;
    default: k_link_substep<DIM, NRHS, 8><<<grid, kBlock, 0, s.stream>>>(A, s.prm); break;
  }
  MTS_LAUNCH_CHECK();
}

// One substep j of the unit-load responses over the region rows.
// u_in/u_out/v/a: [N][nrhs][dim].
void link_substep(Solver &s, int j, const double *u_in, double *u_out, double *v, double *a, const int32_t *ccolor,
                  const int32_t *rhs_color, const int32_t *rhs_dir, int nrhs, const int32_t *slice_layer) {
  if (!s.rsell.n_rows) return;
  LinkArgs A{};
  A.xrec = s.xu[0];
  A.N = s.N;
  A.n_rows = s.rsell.n_rows;
  A.n_slices = s.rsell.n_slices;
  A.T = s.rsell.T;
  A.rows = s.rsell.rows;
  A.slice_layer = slice_layer ? slice_layer : s.rsell.slice_layer;
  A.jmax = j - 1;
  A.col = s.rsell.col;
  A.coef = s.rsell.coef;
  A.mask = s.rsell.mask;
  A.mass = s.mass;
  A.u_in = u_in;
  A.u_out = u_out;
  A.v = v;
  A.a = a;
  A.cidx = s.cidx;
  A.ccolor = ccolor;
  for (int b = 0; b < nrhs; b++) {
    A.rhs_color[b] = rhs_color[b];
    A.rhs_dir[b] = rhs_dir[b];
  }
  A.lfac = (double)j / (double)s.m;
  A.first = j == 1 ? 1 : 0;
  if (s.dim == 2) {
    if (nrhs != 8) throw ArgError{"link batch must hold 8 right-hand sides in 2D"};
    launch_link<2, 8>(s, A);
  } else {
    if (nrhs != 6) throw ArgError{"link batch must hold 6 right-hand sides in 3D"};
    launch_link<3, 6>(s, A);
  }
}

void link_records_init(Solver &s) {
  for (int k = 0; k < 2; k++) {
    k_link_records<<<nblk(s.N), 256, 0, s.stream>>>(s.x, s.N, s.dim, s.Wxu[k]);
    MTS_LAUNCH_CHECK();
  }
}

// Substep j of the final update's response with multipliers s.lam: reads
// records Wxu[k], writes Wxu[k ^ 1]; the last substep (add) adds W_m into the
// PD state.
void link_final_substep(Solver &s, int j, int k, bool add, int side, int snap_slot) {
  if (!s.rsell.n_rows) return;
  Link1Args A{};
  A.N = s.N;
  A.n_rows = s.rsell.n_rows;
  A.n_slices = s.rsell.n_slices;
  A.T = s.rsell.T;
  A.rows = s.rsell.rows;
  A.slice_layer = s.rsell.slice_layer;
  A.jmax = j - 1;
  A.slots = s.rsell.slots;
  A.mask = s.rsell.mask;
  A.mass = s.mass;
  A.w_in = s.Wxu[k];
  A.w_out = s.Wxu[k ^ 1];
  A.v = s.Wv;
  A.a = s.Wa;
  A.cidx = s.cidx;
  A.lam = s.lam;
  A.lfac = (double)j / (double)s.m;
  A.first = j == 1 ? 1 : 0;
  A.add = add ? 1 : 0;
  if (add) {
    A.Uxu = s.xu[s.cur];
    A.Uxu_pred = s.xu[s.cur ^ 1];
    A.Uv = s.v;
    A.Ua = s.a;
  }
  const bool halo = s.rsell.halo_max > 0;
  unsigned grid = (unsigned)((A.n_slices * WAVE + kBlock - 1) / kBlock);
  size_t shm = 0;
  if (halo) {  // the slot records hold LDS offsets: the staged kernel is the only one that reads them
    A.wg_start = s.rsell.wg_start;
    A.halo_off = s.rsell.halo_off;
    A.halo_ids = s.rsell.halo_ids;
    grid = (unsigned)s.rsell.n_wg;
    shm = (size_t)s.rsell.halo_max * 16 * s.dim;
  }
  A.n_link_blocks = grid;
  A.side = side;
  int64_t side_threads = 0;
  if (side == kSideRing) {
    A.ring = fe_ring_args(s);
    side_threads = s.n_ring * WAVE;
  } else if (side == kSideElem) {
    A.elem = fe_elem_args(s, true);
    side_threads = s.ne;
  } else if (side == kSideGather) {
    A.gather = fe_gather_args(s);
    side_threads = s.nfe;
  } else if (side == kSideSnap) {
    A.snap_src = s.sell.mask;
    A.snap_dst = s.mask_snap[snap_slot];
    A.snap_n = s.sell.n_words;
    A.snap_flag = s.region_flag;
    side_threads = std::max<int64_t>(s.sell.n_words, 1);
  }
  grid += (unsigned)((side_threads + kBlock - 1) / kBlock);
#define MTS_LF(D, LL)                                                                        \
  do {                                                                                       \
    if (halo) k_link_final<D, LL, true><<<grid, kBlock, shm, s.stream>>>(A, s.prm);          \
    else k_link_final<D, LL, false><<<grid, kBlock, 0, s.stream>>>(A, s.prm);                \
  } while (0)
  if (s.dim == 2) {
    switch (s.rsell.L) {
      case 1: MTS_LF(2, 1); break;
      case 2: MTS_LF(2, 2); break;
      case 4: MTS_LF(2, 4); break;
      default: MTS_LF(2, 8); break;
    }
  } else {
    switch (s.rsell.L) {
      case 1: MTS_LF(3, 1); break;
      case 2: MTS_LF(3, 2); break;
      case 4: MTS_LF(3, 4); break;
      default: MTS_LF(3, 8); break;
    }
  }
#undef MTS_LF
  MTS_LAUNCH_CHECK();
}


}  // namespace mts
