// Sliced-ELL bond layout for the bond pass: neighbour indices, bond-state words
// (pre-crack bonds start broken, i.e. Eq. 4 with an already-exceeded history)
// and the per-bond coefficient w_ik c(|xi_ik|) V_i V_k of Eq. 2 with the
// Arlequin bond weight w_ik = 1 - (alpha_i + alpha_k)/2.
#include <algorithm>

#include "device_math.h"

namespace mts {

namespace {

constexpr int kThreads = 256;
inline unsigned blocks_for(int64_t n, int t = kThreads) { return (unsigned)((n + t - 1) / t); }

struct Cracks {
  int n;
  double c[8][3];
};

// Pre-crack (horizontal segment y = yc, x_start <= x* <= x_end, tip inclusive);
// x* from the endpoint with the smaller id so both directions agree.
__device__ inline bool crosses_crack(const double *x, int64_t N, int64_t i, int64_t k, const Cracks &cr) {
  int64_t p = i < k ? i : k, q = i < k ? k : i;
  double xp = x[p], yp = x[N + p], xq = x[q], yq = x[N + q];
  for (int c = 0; c < cr.n; c++) {
    double yc = cr.c[c][0];
    if ((yp - yc) * (yq - yc) < 0.0) {
      double xs = xp + (yc - yp) * (xq - xp) / (yq - yp);
      if (xs >= cr.c[c][1] && xs <= cr.c[c][2]) return true;
    }
  }
  return false;
}

__global__ void k_slice_width(const int32_t *rows, int64_t n_rows, const int32_t *rp, int L, int32_t *width,
                              int64_t n_slices) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_slices) return;
  const int S = WAVE / L;
  int w = 0;
  for (int j = 0; j < S; j++) {
    int64_t r = s * S + j;
    if (r >= n_rows) break;
    int64_t i = rows[r];
    int len = rp[i + 1] - rp[i];
    w = len > w ? len : w;
  }
  width[s] = ((w + L - 1) / L) * L;
}

// One thread per (slice, lane).
__global__ void k_sell_fill(const int32_t *rows, int64_t n_rows, int64_t n_slices, const int32_t *rp,
                            const int32_t *csr_col, int L, const int32_t *width, const int64_t *slot_off,
                            int32_t *col) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t s = g / WAVE;
  if (s >= n_slices) return;
  int lane = (int)(g % WAVE);
  const int S = WAVE / L;
  int j = lane / L, l = lane % L;
  int64_t r = s * S + j;
  int T = width[s] / L;
  int64_t i = r < n_rows ? rows[r] : -1;
  int len = i >= 0 ? rp[i + 1] - rp[i] : 0;
  for (int t = 0; t < T; t++) {
    int k = t * L + l;
    int32_t v = 0;
    if (i >= 0) v = k < len ? csr_col[rp[i] + k] : (int32_t)i;
    col[slot_off[s] + (int64_t)t * WAVE + lane] = v;
  }
}

// One thread per (slice, t) word.  src_mask == nullptr: initial states from the
// crack segments; otherwise bits gathered from the full-lattice layout.
__global__ void k_sell_mask(const int32_t *rows, int64_t n_rows, int64_t n_slices, const int32_t *rp,
                            const int32_t *csr_col, int L, const int32_t *width, const int64_t *word_off,
                            uint64_t *mask, const double *x, int64_t N, int dim, Cracks cr,
                            const uint64_t *src_mask, const int64_t *src_word_off, int src_L, const int32_t *src_row_of) {
  int64_t s = blockIdx.y;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_slices || t >= width[s] / L) return;
  const int S = WAVE / L;
  uint64_t word = 0;
  for (int lane = 0; lane < WAVE; lane++) {
    int j = lane / L, l = lane % L;
    int64_t r = s * S + j;
    if (r >= n_rows) break;
    int64_t i = rows[r];
    int len = rp[i + 1] - rp[i];
    int k = t * L + l;
    if (k >= len) continue;
    bool intact;
    if (src_mask) {
      intact = full_bit(src_word_off, src_mask, src_L, src_row_of ? src_row_of[i] : i, k);
    } else {
      int64_t c = csr_col[rp[i] + k];
      intact = !(dim == 2 && crosses_crack(x, N, i, c, cr));
    }
    if (intact) word |= 1ull << lane;
  }
  mask[word_off[s] + t] = word;
}

// Per-bond coefficient ((w_ik c(r)) V_i V_k) for the fused bond pass; the
// mixed form stores coef / m_i in single precision.
__global__ void k_sell_coef(const int32_t *rows, int64_t n_rows, int64_t n_slices, const int32_t *rp,
                            const int32_t *csr_col, int L, const int32_t *width, const int64_t *slot_off,
                            const double *x, int64_t N, const double *alpha, const double *mass, Params P,
                            double *coef, float *coef32) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t s = g / WAVE;
  if (s >= n_slices) return;
  int lane = (int)(g % WAVE);
  const int S = WAVE / L;
  int j = lane / L, l = lane % L;
  int64_t r = s * S + j;
  int T = width[s] / L;
  int64_t i = r < n_rows ? rows[r] : -1;
  int len = i >= 0 ? rp[i + 1] - rp[i] : 0;
  for (int t = 0; t < T; t++) {
    int k = t * L + l;
    double cf = 0.0;
    if (i >= 0 && k < len) {
      int64_t c = csr_col[rp[i] + k];
      double d0 = x[c] - x[i], d1 = x[N + c] - x[N + i];
      double r2 = d0 * d0 + d1 * d1;
      if (P.dim == 3) {
        double d2 = x[2 * N + c] - x[2 * N + i];
        r2 = r2 + d2 * d2;
      }
      double w = 1.0 - 0.5 * (alpha[i] + alpha[c]);
      cf = ((w * cfun(P, sqrt(r2))) * P.VV);
    }
    int64_t pos = slot_off[s] + (int64_t)t * WAVE + lane;
    if (coef) coef[pos] = cf;
    if (coef32) coef32[pos] = (float)(i >= 0 ? cf / mass[i] : 0.0);
  }
}

__global__ void k_mask_to_csr(int64_t N, const int32_t *rp, const int64_t *word_off, const uint64_t *mask, int L,
                              const int32_t *row_of, uint8_t *out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int len = rp[i + 1] - rp[i];
  const int64_t r = row_of ? row_of[i] : i;
  for (int k = 0; k < len; k++) out[rp[i] + k] = (uint8_t)full_bit(word_off, mask, L, r, k);
}

__global__ void k_damage(int64_t N, const int32_t *rp, const int64_t *word_off, const uint64_t *mask, int L,
                         const int32_t *row_of, double *phi) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int len = rp[i + 1] - rp[i];
  const int64_t r = row_of ? row_of[i] : i;
  int cnt = 0;
  for (int k = 0; k < len; k++) cnt += (int)full_bit(word_off, mask, L, r, k);
  phi[i] = len > 0 ? 1.0 - (double)cnt / (double)len : 0.0;  // Eq. 5, uniform nodal volumes
}

}  // namespace

void build_sell(Solver &s, Sell &out, const std::vector<int32_t> &rows_host, const uint64_t *src_mask_full, int L) {
  hipStream_t st = s.stream;
  DeviceArena &ar = s.arena;
  out.L = L;
  const int S = WAVE / L;
  out.n_rows = (int64_t)rows_host.size();
  out.n_slices = (out.n_rows + S - 1) / S;
  int64_t ns = out.n_slices;
  out.rows = ar.alloc<int32_t>(out.n_rows);
  if (out.n_rows)
    MTS_HIP(hipMemcpyAsync(out.rows, rows_host.data(), sizeof(int32_t) * out.n_rows, hipMemcpyHostToDevice, st));
  out.width = ar.alloc<int32_t>(ns);
  if (ns) {
    k_slice_width<<<blocks_for(ns), kThreads, 0, st>>>(out.rows, out.n_rows, s.rp, L, out.width, ns);
    MTS_LAUNCH_CHECK();
  }
  std::vector<int32_t> w(ns);
  if (ns) MTS_HIP(hipMemcpyAsync(w.data(), out.width, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, st));
  MTS_HIP(hipStreamSynchronize(st));
  // One width for every slice (the largest family, rounded up to L): the bond
  // pass then computes slice offsets instead of loading them.  Families shorter
  // than the width are padded with state-0 slots.
  int maxw = 0;
  for (int64_t q = 0; q < ns; q++) maxw = std::max(maxw, (int)w[q]);
  for (int64_t q = 0; q < ns; q++) w[q] = maxw;
  if (ns) MTS_HIP(hipMemcpyAsync(out.width, w.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, st));
  out.T = maxw / L;
  std::vector<int64_t> so(ns + 1), wo(ns + 1);
  so[0] = wo[0] = 0;
  int maxt = 0;
  for (int64_t q = 0; q < ns; q++) {
    so[q + 1] = so[q] + (int64_t)(w[q] / L) * WAVE;
    wo[q + 1] = wo[q] + w[q] / L;
    maxt = std::max(maxt, w[q] / L);
  }
  out.n_slots = so[ns];
  out.n_words = wo[ns];
  out.slot_off = ar.alloc<int64_t>(ns + 1);
  out.word_off = ar.alloc<int64_t>(ns + 1);
  MTS_HIP(hipMemcpyAsync(out.slot_off, so.data(), sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemcpyAsync(out.word_off, wo.data(), sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice, st));
  // kSpareIters iterations of zeros past the last slice keep unrolled loads in bounds
  out.col = ar.alloc<int32_t>(out.n_slots + kSpareIters * WAVE);
  out.mask = ar.alloc<uint64_t>(out.n_words + kSpareIters);
  MTS_HIP(hipMemsetAsync(out.col, 0, sizeof(int32_t) * (out.n_slots + kSpareIters * WAVE), st));
  MTS_HIP(hipMemsetAsync(out.mask, 0, sizeof(uint64_t) * (out.n_words + kSpareIters), st));
  if (ns) {
    k_sell_fill<<<blocks_for(ns * WAVE), kThreads, 0, st>>>(out.rows, out.n_rows, ns, s.rp, s.csr_col, L, out.width,
                                                            out.slot_off, out.col);
    MTS_LAUNCH_CHECK();
    Cracks cr{};
    cr.n = s.p.n_cracks;
    for (int c = 0; c < cr.n; c++)
      for (int q = 0; q < 3; q++) cr.c[c][q] = s.p.cracks[c][q];
    if (maxt > 0) {
      dim3 grid((unsigned)((maxt + 63) / 64), (unsigned)ns);
      k_sell_mask<<<grid, 64, 0, st>>>(out.rows, out.n_rows, ns, s.rp, s.csr_col, L, out.width, out.word_off,
                                       out.mask, s.x, s.N, s.dim, cr, src_mask_full, s.sell.word_off, s.sell.L,
                                       s.sell.row_of);
      MTS_LAUNCH_CHECK();
    }
  }
  MTS_HIP(hipStreamSynchronize(st));
}

void sell_regather_mask(Solver &s, Sell &out, const uint64_t *src_mask_full) {
  if (!out.n_slices) return;
  std::vector<int32_t> w(out.n_slices);
  MTS_HIP(hipMemcpyAsync(w.data(), out.width, sizeof(int32_t) * out.n_slices, hipMemcpyDeviceToHost, s.stream));
  MTS_HIP(hipStreamSynchronize(s.stream));
  int maxt = 0;
  for (int32_t v : w) maxt = std::max(maxt, (int)v / out.L);
  if (!maxt) return;
  Cracks cr{};
  dim3 grid((unsigned)((maxt + 63) / 64), (unsigned)out.n_slices);
  k_sell_mask<<<grid, 64, 0, s.stream>>>(out.rows, out.n_rows, out.n_slices, s.rp, s.csr_col, out.L, out.width,
                                          out.word_off, out.mask, s.x, s.N, s.dim, cr, src_mask_full,
                                          s.sell.word_off, s.sell.L, s.sell.row_of);
  MTS_LAUNCH_CHECK();
}

void sell_coefficients(Solver &s, Sell &out) {
  if (!out.n_slices) return;
  bool mixed = s.precision == MTS_MIXED;
  const int64_t ns = out.n_slots + kSpareIters * WAVE;
  if (!out.coef) {
    out.coef = s.arena.alloc<double>(ns);
    MTS_HIP(hipMemsetAsync(out.coef, 0, sizeof(double) * ns, s.stream));
  }
  if (mixed && !out.coef32) {
    out.coef32 = s.arena.alloc<float>(ns);
    MTS_HIP(hipMemsetAsync(out.coef32, 0, sizeof(float) * ns, s.stream));
  }
  k_sell_coef<<<blocks_for(out.n_slices * WAVE), kThreads, 0, s.stream>>>(
      out.rows, out.n_rows, out.n_slices, s.rp, s.csr_col, out.L, out.width, out.slot_off, s.x, s.N, s.alpha,
      s.mass, s.prm, out.coef, mixed ? out.coef32 : nullptr);
  MTS_LAUNCH_CHECK();
}

namespace {
// Slot records {byte offset of the neighbour's node record, coefficient}
// (FP64: coefficient first, then the offset); the
// offset is col * rb (rb = bytes of one record), in the record array or, when
// the records are staged, in the workgroup's LDS list.
__global__ void k_pack_slots(int64_t n, const int32_t *col, uint32_t rb, const double *coef, const float *coef32,
                             uint32_t *slots) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t off = (uint32_t)col[p] * rb;
  if (coef32) {
    slots[2 * p] = off;
    slots[2 * p + 1] = __float_as_uint(coef32[p]);
  } else {
    // coefficient first: it lands in an aligned register pair when loaded
    const uint64_t b = (uint64_t)__double_as_longlong(coef[p]);
    slots[3 * p] = (uint32_t)b;
    slots[3 * p + 1] = (uint32_t)(b >> 32);
    slots[3 * p + 2] = off;
  }
}
}  // namespace

namespace {
// Mixed-form slot records of the staged pass, one per two iterations of a
// lane: {coef32(t), coef32(t + 1), idx(t) | idx(t + 1) << 16}, idx being the
// neighbour's position in the workgroup's LDS list.  Record (slice, pair P,
// lane) sits at (slice * TP + P) * 64 + lane; an odd T leaves the second half
// of the last pair empty, and kSpareIters * 64 empty records follow.
__global__ void k_pack_pairs(int64_t n_rec, int64_t n_real, int T, int TP, const int32_t *local, const float *coef32,
                             uint32_t *rec) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rec) return;
  uint32_t c0 = 0u, c1 = 0u, ix = 0u;
  if (r < n_real) {
    const int64_t lane = r % WAVE, g = r / WAVE, sl = g / TP, pr = g % TP;
    const int t0 = (int)(2 * pr);
    const int64_t p0 = (sl * T + t0) * WAVE + lane;
    c0 = __float_as_uint(coef32[p0]);
    ix = (uint32_t)local[p0];
    if (t0 + 1 < T) {
      c1 = __float_as_uint(coef32[p0 + WAVE]);
      ix |= (uint32_t)local[p0 + WAVE] << 16;
    }
  }
  rec[3 * r] = c0;
  rec[3 * r + 1] = c1;
  rec[3 * r + 2] = ix;
}
}  // namespace

void sell_pack_pairs(Solver &s, Sell &out, const int32_t *dev_local) {
  const int T = out.T, TP = (T + 1) / 2;
  const int64_t n_real = out.n_slices * TP * WAVE, n_rec = n_real + kSpareIters * WAVE;
  // the unpaired records are not needed any more: free them first (lower peak)
  if (out.slots) s.arena.release(out.slots);
  uint32_t *rec = s.arena.alloc<uint32_t>((size_t)n_rec * 3);
  k_pack_pairs<<<blocks_for(n_rec), kThreads, 0, s.stream>>>(n_rec, n_real, T, TP, dev_local, out.coef32, rec);
  MTS_LAUNCH_CHECK();
  out.slots = rec;
  out.pair_slots = true;
}

void sell_pack_slots(Solver &s, Sell &out, const int32_t *dev_col, bool fp64) {
  const bool mixed = !fp64 && !out.fp64_slots && s.precision == MTS_MIXED;
  const int64_t n = out.n_slots + kSpareIters * WAVE;
  if (!out.slots) out.slots = s.arena.alloc<uint32_t>((size_t)n * (mixed ? 2 : 3));
  k_pack_slots<<<blocks_for(n), kThreads, 0, s.stream>>>(n, dev_col ? dev_col : out.col, 16u * (uint32_t)s.dim, out.coef,
                                                          mixed ? out.coef32 : nullptr, out.slots);
  MTS_LAUNCH_CHECK();
}

// Per-workgroup neighbour lists for LDS staging (host side, integer work only).
// Workgroups take consecutive slices, at most G = wg_waves each, and a new one
// starts where a slice's first row lies in another spatial tile, so that a
// workgroup covers one tile.  Its list is the sorted set of every node its
// slots name (padding slots name node 0).  Staging is used only when every
// list fits the LDS share of one workgroup (64 KiB for 4 wavefronts, 80 KiB
// for 8: two such workgroups per CU).
void sell_build_halo(Solver &s, Sell &out) {
  const int G = out.wg_waves;
  int dev = 0, lds_max = 65536;
  MTS_HIP(hipGetDevice(&dev));
  MTS_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  const int kHaloMax = std::min(G == 8 ? 81920 : 65536, lds_max) / (16 * s.dim);  // records that fit (< 2^16)
  out.halo_max = 0;
  if (!out.n_slices) return;
  hipStream_t st = s.stream;
  const int64_t n = out.n_slots + kSpareIters * WAVE;
  std::vector<int32_t> col(n);
  MTS_HIP(hipMemcpyAsync(col.data(), out.col, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
  MTS_HIP(hipStreamSynchronize(st));
  const int64_t per_slice = (int64_t)out.T * WAVE;
  const int64_t S = WAVE / out.L;  // rows per slice
  std::vector<int32_t> start{0};
  for (int64_t sl = 1; sl < out.n_slices; sl++) {
    const bool full = sl - start.back() == G;
    const bool new_tile = !out.h_tile.empty() && out.h_tile[sl * S] != out.h_tile[start.back() * S];
    if (full || new_tile) start.push_back((int32_t)sl);
  }
  start.push_back((int32_t)out.n_slices);
  const int64_t nwg = (int64_t)start.size() - 1;
  std::vector<int32_t> off(nwg + 1, 0), ids, pos_of(s.N, -1), local(n, 0);
  std::vector<int64_t> stamp(s.N, -1);
  std::vector<int32_t> set;
  int hmax = 0;
  for (int64_t w = 0; w < nwg; w++) {
    const int64_t a = start[w] * per_slice, b = start[w + 1] * per_slice;
    set.clear();
    for (int64_t q = a; q < b; q++) {
      const int32_t c = col[q];
      if (stamp[c] != w) {
        stamp[c] = w;
        set.push_back(c);
      }
    }
    std::sort(set.begin(), set.end());
    hmax = std::max(hmax, (int)set.size());
    if (hmax > kHaloMax) return;  // too spread out: gather from global memory instead
    for (size_t h = 0; h < set.size(); h++) pos_of[set[h]] = (int32_t)h;
    for (int64_t q = a; q < b; q++) local[q] = pos_of[col[q]];
    ids.insert(ids.end(), set.begin(), set.end());
    off[w + 1] = (int32_t)ids.size();
  }
  // Dependencies between workgroups: w depends on the owners of the nodes its
  // list holds, and (symmetric closure) on the workgroups whose lists hold w's
  // rows.  Rows outside this layout (link region) have no owner.
  {
    std::vector<int32_t> rows_h(out.n_rows);
    MTS_HIP(hipMemcpyAsync(rows_h.data(), out.rows, sizeof(int32_t) * out.n_rows, hipMemcpyDeviceToHost, st));
    MTS_HIP(hipStreamSynchronize(st));
    std::vector<int32_t> owner(s.N, -1);
    for (int64_t w = 0; w < nwg; w++)
      for (int64_t r = start[w] * S; r < std::min<int64_t>(start[w + 1] * S, out.n_rows); r++) owner[rows_h[r]] = (int32_t)w;
    std::vector<std::pair<int32_t, int32_t>> pairs;
    for (int64_t w = 0; w < nwg; w++)
      for (int32_t h = off[w]; h < off[w + 1]; h++) {
        const int32_t o = owner[ids[h]];
        if (o >= 0 && o != w) {
          pairs.push_back({(int32_t)w, o});
          pairs.push_back({o, (int32_t)w});
        }
      }
    std::sort(pairs.begin(), pairs.end());
    pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
    std::vector<int32_t> doff(nwg + 1, 0), dids(pairs.size());
    for (size_t k = 0; k < pairs.size(); k++) {
      doff[pairs[k].first + 1]++;
      dids[k] = pairs[k].second;
    }
    for (int64_t w = 0; w < nwg; w++) {
      out.max_deps = std::max(out.max_deps, doff[w + 1]);
      doff[w + 1] += doff[w];
    }
    out.dep_off = s.arena.alloc<int32_t>(nwg + 1);
    out.dep_ids = s.arena.alloc<int32_t>(std::max<size_t>(dids.size(), 1));
    out.wg_flag = s.arena.alloc<uint32_t>(nwg);
    MTS_HIP(hipMemcpyAsync(out.dep_off, doff.data(), sizeof(int32_t) * (nwg + 1), hipMemcpyHostToDevice, st));
    if (!dids.empty())
      MTS_HIP(hipMemcpyAsync(out.dep_ids, dids.data(), sizeof(int32_t) * dids.size(), hipMemcpyHostToDevice, st));
    MTS_HIP(hipMemsetAsync(out.wg_flag, 0, sizeof(uint32_t) * nwg, st));
    MTS_HIP(hipStreamSynchronize(st));
  }
  out.n_wg = nwg;
  out.wg_start = s.arena.alloc<int32_t>(nwg + 1);
  MTS_HIP(hipMemcpyAsync(out.wg_start, start.data(), sizeof(int32_t) * (nwg + 1), hipMemcpyHostToDevice, st));
  out.halo_off = s.arena.alloc<int32_t>(nwg + 1);
  out.halo_ids = s.arena.alloc<int32_t>(std::max<size_t>(ids.size(), 1));
  int32_t *dlocal = s.arena.alloc<int32_t>(n);
  MTS_HIP(hipMemcpyAsync(out.halo_off, off.data(), sizeof(int32_t) * (nwg + 1), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemcpyAsync(out.halo_ids, ids.data(), sizeof(int32_t) * ids.size(), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemcpyAsync(dlocal, local.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
  // the mixed form's staged pass reads paired records with 16-bit list positions
  if (!out.fp64_slots && s.precision == MTS_MIXED) sell_pack_pairs(s, out, dlocal);
  else sell_pack_slots(s, out, dlocal);
  MTS_HIP(hipStreamSynchronize(st));
  s.arena.release(dlocal);
  out.halo_max = hmax;
}

void bonds_to_csr_state(Solver &s, uint8_t *dev_out) {
  k_mask_to_csr<<<blocks_for(s.N), kThreads, 0, s.stream>>>(s.N, s.rp, s.sell.word_off, s.sell.mask, s.sell.L,
                                                            s.sell.row_of, dev_out);
  MTS_LAUNCH_CHECK();
}

void pd_damage(Solver &s) {
  k_damage<<<blocks_for(s.N), kThreads, 0, s.stream>>>(s.N, s.rp, s.sell.word_off, s.sell.mask, s.sell.L,
                                                       s.sell.row_of, s.damage);
  MTS_LAUNCH_CHECK();
}

}  // namespace mts
