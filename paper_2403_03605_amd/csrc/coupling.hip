// Arlequin coupling with velocity-continuity multipliers across the overlap and
// the multi-time-step free/link split (Sec. 2.5, Eq. 41-50, Algorithm 1).
//
// Constraints sit at every PD node with alpha > 0; G_P is Boolean and the rows
// of G_F interpolate the FE velocity at the PD node (N_a(x_p)).  The multiplier
// matrix H = G_P Ydot^PD_m + 1/2 dt_FE G_F M_F^-1 G_F^T is assembled from link
// runs (m substeps of the linear PD response to a unit multiplier ramp, no
// breaking) batched over colour classes of constraints whose supports do not
// overlap, then inverted once.  Every macro step solves H lambda_m = G_F v~_F -
// G_P V_m and applies U = V + Y lambda_m, the PD part by re-running the link
// problem with the actual multipliers over the region the response can reach
// ((m-1) horizons from the constraints), which equals Y^PD lambda_m.
#include "internal.h"

#include <algorithm>
#include <map>
#include <cmath>
#include <unordered_map>

namespace mts {

void link_substep(Solver &s, int j, const double *u_in, double *u_out, double *v, double *a, const int32_t *ccolor,
                  const int32_t *rhs_color, const int32_t *rhs_dir, int nrhs, const int32_t *slice_layer);
void link_records_init(Solver &s);
void link_final_substep(Solver &s, int j, int k, bool add, int side, int snap_slot);
void sell_regather_mask(Solver &s, Sell &out, const uint64_t *src_mask_full);

namespace {

inline unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

__device__ inline double shape_c(int dim, int a, const double *xi) {
  const int q4[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};
  double v = (dim == 2 ? 0.25 : 0.125) * (1.0 + q4[a & 3][0] * xi[0]) * (1.0 + q4[a & 3][1] * xi[1]);
  if (dim == 3) v = v * (1.0 + (a < 4 ? -1.0 : 1.0) * xi[2]);
  return v;
}

// Element containing each constraint node and the interpolation weights N_a(x_p).
__global__ void k_gf(int64_t nc, int dim, int nen, const int32_t *cn, const double *x, int64_t N, double lo0,
                     double lo1, double lo2, double h, int64_t ne0, int64_t ne1, int64_t ne2, int32_t *cel,
                     double *cw) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc) return;
  int64_t i = cn[q];
  double lo[3] = {lo0, lo1, lo2};
  int64_t nen_ax[3] = {ne0, ne1, ne2};
  int64_t ei[3] = {0, 0, 0};
  double xi[3] = {0, 0, 0};
  for (int a = 0; a < dim; a++) {
    double t = (x[a * N + i] - lo[a]) / h;
    ei[a] = (int64_t)floor(t);
    if (ei[a] >= nen_ax[a]) ei[a] = nen_ax[a] - 1;
    if (ei[a] < 0) ei[a] = 0;
    xi[a] = 2.0 * (t - (double)ei[a]) - 1.0;
  }
  int64_t e = (ei[2] * ne1 + ei[1]) * ne0 + ei[0];
  cel[q] = (int32_t)e;
  for (int a = 0; a < nen; a++) {
    double v;
    if (dim == 2) {
      const int q4[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};
      v = 0.25 * (1.0 + q4[a][0] * xi[0]) * (1.0 + q4[a][1] * xi[1]);
    } else {
      v = shape_c(3, a, xi);
    }
    cw[q * nen + a] = v;
  }
}

// Link region: nodes within (m-1) horizons of a constraint node (the reach of
// the unit-load responses).  layer: smallest h with a constraint within h
// horizons (slightly generous), used to skip rows whose link state is still
// exactly zero at a given link substep.
__global__ void k_region(const double *x, int64_t N, int dim, const int32_t *cn, int64_t nc, double R2,
                         double delta, int m, uint8_t *flag, int32_t *layer) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double best = 1e300;
  for (int64_t q = 0; q < nc; q++) {
    int64_t c = cn[q];
    double d0 = x[i] - x[c];
    double d1 = x[N + i] - x[N + c];
    double r2 = d0 * d0 + d1 * d1;
    if (dim == 3) {
      double d2 = x[2 * N + i] - x[2 * N + c];
      r2 = r2 + d2 * d2;
    }
    best = r2 < best ? r2 : best;
  }
  flag[i] = best <= R2 ? 1 : 0;
  int h = m;
  for (int k = m - 1; k >= 0; k--) {
    double hk = (double)k * delta;
    if (best <= hk * hk * (1.0 + 1e-9)) h = k;
  }
  layer[i] = h;
}

__global__ void k_slice_layer(const int32_t *rows, int64_t n_rows, int64_t n_slices, int L, const int32_t *layer,
                              int32_t *slice_layer) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_slices) return;
  const int S = WAVE / L;
  int h = 1 << 30;
  for (int j = 0; j < S; j++) {
    int64_t r = s * S + j;
    if (r >= n_rows) break;
    int v = layer[rows[r]];
    h = v < h ? v : h;
  }
  slice_layer[s] = h;
}

// Layer of every slice of the link region with respect to the constraint
// nodes loaded by one batch of unit loads: the smallest k <= m such that some
// row of the slice lies within k horizons of a loaded node (m if none).  A
// response that has run j substeps is still exactly zero beyond j - 1 such
// horizons, so the batch's link substeps skip those slices.
__global__ __launch_bounds__(WAVE) void k_batch_layer(const double *x, int64_t N, int dim, const int32_t *rows,
                                                       int64_t n_rows, int64_t n_slices, int L, const int32_t *nodes,
                                                       int n_nodes, double delta, int m, int32_t *slice_layer) {
  // one wavefront per slice: the lanes split the (row, loaded node) pairs and
  // the smallest squared distance is combined across the wavefront (min is exact)
  const int64_t s = blockIdx.x;
  if (s >= n_slices) return;
  const int lane = (int)threadIdx.x;
  const int S = WAVE / L;
  const int nr = (int)std::min<int64_t>(S, n_rows - s * S);
  double best = 1e300;
  for (int e = lane; e < nr * n_nodes; e += WAVE) {
    const int64_t i = rows[s * S + e / n_nodes];
    const int64_t c = nodes[e % n_nodes];
    const double d0 = x[i] - x[c];
    const double d1 = x[N + i] - x[N + c];
    double r2 = d0 * d0 + d1 * d1;
    if (dim == 3) {
      const double d2 = x[2 * N + i] - x[2 * N + c];
      r2 = r2 + d2 * d2;
    }
    best = r2 < best ? r2 : best;
  }
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const double t = __shfl_xor(best, o, WAVE);
    best = t < best ? t : best;
  }
  if (lane != 0) return;
  int h = m;
  for (int k = m - 1; k >= 0; k--) {
    const double hk = (double)k * delta;
    if (best <= hk * hk * (1.0 + 1e-9)) h = k;
  }
  slice_layer[s] = h;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_set_cidx(const int32_t *cn, int64_t nc, int32_t *cidx) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nc) cidx[cn[q]] = (int32_t)q;
}

// H[(q, d'), (p, dir)] = velocity d' of RHS b at node q (responses node-major,
// [N][nrhs][dim]) for the loaded constraint p of RHS b that owns q (the only
// loaded node whose response can reach q).
// csel (or nullptr for all): only the columns of the constraints this rebuild loaded.
__global__ void k_extract(int64_t nc, int dim, int64_t nl, int nrhs, const int32_t *cn, const int32_t *owner,
                          const int32_t *rhs_color, const int32_t *rhs_dir, const double *Wv, const uint8_t *csel,
                          double *H) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc) return;
  int64_t node = cn[q];
  for (int b = 0; b < nrhs; b++) {
    int c = rhs_color[b];
    if (c < 0) continue;
    int32_t p = owner[(int64_t)c * nc + q];
    if (p < 0 || (csel && !csel[p])) continue;
    for (int d = 0; d < dim; d++)
      H[(q * dim + d) * nl + (int64_t)p * dim + rhs_dir[b]] = Wv[(node * nrhs + b) * dim + d];
  }
}

// + 1/2 dt_FE G_F M_F^-1 G_F^T (prescribed-velocity dofs do not respond).
__global__ void k_add_hf(int64_t nc, int dim, int nen, int64_t nl, const int32_t *cel, const int32_t *conn,
                         const double *cw, const double *mF, const uint8_t *bc, double hdtF, int64_t ne0,
                         int64_t ne1, const uint8_t *csel, double *H) {
  int64_t pq = (int64_t)blockIdx.y * blockDim.y + threadIdx.y;
  int64_t qq = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pq >= nc || qq >= nc || (csel && !csel[qq])) return;
  int64_t ep = cel[pq], eq = cel[qq];
  int64_t dx = ep % ne0 - eq % ne0, dy = (ep / ne0) % ne1 - (eq / ne0) % ne1, dz = ep / (ne0 * ne1) - eq / (ne0 * ne1);
  if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1) return;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int ap = 0; ap < nen; ap++)
    for (int aq = 0; aq < nen; aq++) {
      int64_t np_ = conn[ep * nen + ap], nq_ = conn[eq * nen + aq];
      if (np_ != nq_) continue;
      for (int d = 0; d < dim; d++) {
        if (bc[np_ * dim + d]) continue;
        acc[d] += cw[pq * nen + ap] * cw[qq * nen + aq] / mF[np_];
      }
    }
  for (int d = 0; d < dim; d++) H[(pq * dim + d) * nl + qq * dim + d] += hdtF * acc[d];
}

// H += HF (the implicit FE block, computed once); csel: only those columns
__global__ void k_add_dense(int64_t n, int64_t nl, int dim, const uint8_t *csel, const double *HF, double *H) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (!csel || csel[(i % nl) / dim])) H[i] = H[i] + HF[i];
}

// Columns of the constraints in csel set to zero (before they are recomputed).
__global__ void k_zero_cols(int64_t nl, int dim, const uint8_t *csel, double *H) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nl * nl && csel[(i % nl) / dim]) H[i] = 0.0;
}

// Nodes whose row of the full layout holds a bond whose state differs between
// two masks (one wavefront per slice; bit j * L + l of a word belongs to row j).
__global__ __launch_bounds__(WAVE) void k_dirty_nodes(const int64_t *word_off, int64_t n_slices, const int32_t *rows,
                                                      int64_t n_rows, int L, const uint64_t *a, const uint64_t *b,
                                                      uint8_t *dirty) {
  const int64_t s = blockIdx.x;
  if (s >= n_slices) return;
  const int S = WAVE / L;
  for (int64_t w = word_off[s] + threadIdx.x; w < word_off[s + 1]; w += WAVE) {
    uint64_t d = a[w] ^ b[w];
    while (d) {
      const int bit = __builtin_ctzll(d);
      d &= d - 1;
      const int64_t r = s * S + bit / L;
      if (r < n_rows) dirty[rows[r]] = 1;
    }
  }
}

// r = G_F v~_F - G_P V_m  (right-hand side of Eq. 49, from Eq. 41)
__global__ void k_rhs(int64_t nc, int dim, int nen, const int32_t *cn, const int32_t *cel, const int32_t *conn,
                      const double *cw, const double *vt, const double *vP, int64_t N, double *r,
                      const int32_t *rpos, double *r_blk) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc) return;
  int64_t e = cel[q];
  for (int d = 0; d < dim; d++) {
    double g = 0.0;
    for (int a = 0; a < nen; a++) g += cw[q * nen + a] * vt[(int64_t)conn[e * nen + a] * dim + d];
    const double v = g - vP[d * N + cn[q]];
    r[q * dim + d] = v;
    const int32_t p = rpos[q * dim + d];  // the same entry in the multiplier solve's block order
    if (p >= 0) r_blk[p] = v;
  }
}

}  // namespace

void coupling_setup(Solver &s) {
  const int dim = s.dim;
  const int64_t N = s.N;
  hipStream_t st = s.stream;
  DeviceArena &ar = s.arena;
  // constraint set: PD nodes with alpha > 0 (the overlap)
  std::vector<double> al(N);
  MTS_HIP(hipMemcpyAsync(al.data(), s.alpha, sizeof(double) * N, hipMemcpyDeviceToHost, st));
  MTS_HIP(hipStreamSynchronize(st));
  s.h_cn.clear();
  for (int64_t i = 0; i < N; i++) {
    if (al[i] >= 1.0) throw ArgError{"a PD node has alpha = 1 (zero PD mass)"};
    if (al[i] > 0.0) s.h_cn.push_back((int32_t)i);
  }
  s.nc = (int64_t)s.h_cn.size();
  s.nl = s.nc * dim;
  if (s.nc == 0) throw ArgError{"coupled mode needs an overlap band inside the body"};
  s.cn = ar.alloc<int32_t>(s.nc);
  s.cidx = ar.alloc<int32_t>(N);
  s.cel = ar.alloc<int32_t>(s.nc);
  s.cw = ar.alloc<double>(s.nc * s.nen);
  MTS_HIP(hipMemcpyAsync(s.cn, s.h_cn.data(), sizeof(int32_t) * s.nc, hipMemcpyHostToDevice, st));
  k_fill_i32<<<nb(N), 256, 0, st>>>(s.cidx, N, -1);
  MTS_LAUNCH_CHECK();
  k_set_cidx<<<nb(s.nc), 256, 0, st>>>(s.cn, s.nc, s.cidx);
  MTS_LAUNCH_CHECK();
  k_gf<<<nb(s.nc), 256, 0, st>>>(s.nc, dim, s.nen, s.cn, s.x, N, s.p.dom_lo[0], s.p.dom_lo[1],
                                 dim == 3 ? s.p.dom_lo[2] : 0.0, s.p.fe_h, s.p.fe_n[0], s.p.fe_n[1],
                                 dim == 3 ? s.p.fe_n[2] : 1, s.cel, s.cw);
  MTS_LAUNCH_CHECK();
  std::vector<int32_t> hcel(s.nc);
  std::vector<uint8_t> heact(s.ne);
  MTS_HIP(hipMemcpyAsync(hcel.data(), s.cel, sizeof(int32_t) * s.nc, hipMemcpyDeviceToHost, st));
  MTS_HIP(hipMemcpyAsync(heact.data(), s.eact, s.ne, hipMemcpyDeviceToHost, st));
  MTS_HIP(hipStreamSynchronize(st));
  for (int64_t q = 0; q < s.nc; q++)
    if (!heact[hcel[q]]) throw ArgError{"a constraint node lies in an FE element with zero weight"};
  // FE node -> (constraint * nen + a), ascending constraint order
  std::vector<int32_t> cnt(s.nfe + 1, 0);
  for (int64_t q = 0; q < s.nc; q++)
    for (int a = 0; a < s.nen; a++) cnt[s.h_conn[(int64_t)hcel[q] * s.nen + a] + 1]++;
  for (int64_t n = 0; n < s.nfe; n++) cnt[n + 1] += cnt[n];
  std::vector<int32_t> f2c(cnt[s.nfe]), fill(cnt.begin(), cnt.end() - 1);
  for (int64_t q = 0; q < s.nc; q++)
    for (int a = 0; a < s.nen; a++) f2c[fill[s.h_conn[(int64_t)hcel[q] * s.nen + a]]++] = (int32_t)(q * s.nen + a);
  s.f2c_ptr = ar.alloc<int32_t>(s.nfe + 1);
  s.f2c = ar.alloc<int32_t>(f2c.size());
  MTS_HIP(hipMemcpyAsync(s.f2c_ptr, cnt.data(), sizeof(int32_t) * (s.nfe + 1), hipMemcpyHostToDevice, st));
  if (!f2c.empty())
    MTS_HIP(hipMemcpyAsync(s.f2c, f2c.data(), sizeof(int32_t) * f2c.size(), hipMemcpyHostToDevice, st));
  {
    std::vector<int32_t> ring;
    for (int64_t n = 0; n < s.nfe; n++)
      if (cnt[n + 1] > cnt[n]) ring.push_back((int32_t)n);
    s.n_ring = (int64_t)ring.size();
    s.fe_ring = ar.alloc<int32_t>(ring.size());
    if (!ring.empty())
      MTS_HIP(hipMemcpyAsync(s.fe_ring, ring.data(), sizeof(int32_t) * ring.size(), hipMemcpyHostToDevice, st));
    MTS_HIP(hipStreamSynchronize(st));
  }

  // link region: nodes within (m-1) horizons of a constraint node
  double Rr = (double)(s.m - 1) * s.prm.delta;
  s.in_region = ar.alloc<uint8_t>(N);
  s.layer = ar.alloc<int32_t>(N);
  k_region<<<nb(N), 256, 0, st>>>(s.x, N, dim, s.cn, s.nc, Rr * Rr, s.prm.delta, s.m, s.in_region, s.layer);
  MTS_LAUNCH_CHECK();
  std::vector<uint8_t> reg(N);
  MTS_HIP(hipMemcpyAsync(reg.data(), s.in_region, N, hipMemcpyDeviceToHost, st));
  MTS_HIP(hipStreamSynchronize(st));
  std::vector<int32_t> rrows;
  for (int64_t i = 0; i < N; i++)
    if (reg[i]) rrows.push_back((int32_t)i);
  // with tiled rows the region takes the same spatial tile order, so each
  // workgroup of the final update can stage its neighbours' records in LDS
  const bool region_tiled = s.halo && !s.h_node_tile.empty();
  if (region_tiled)
    std::stable_sort(rrows.begin(), rrows.end(),
                     [&](int32_t a, int32_t b) { return s.h_node_tile[a] < s.h_node_tile[b]; });
  s.n_region = (int64_t)rrows.size();
  build_sell(s, s.rsell, rrows, s.sell.mask,
             s.region_lanes ? s.region_lanes : pick_lanes(s.n_region, s.dim, s.dim == 3 ? ((int64_t)1 << 18) : (int64_t)120000));
  sell_coefficients(s, s.rsell);
  s.rsell.fp64_slots = true;  // the final update runs in FP64 in both forms
  sell_pack_slots(s, s.rsell);
  if (region_tiled && s.rsell.n_slices) {
    s.rsell.h_tile.resize(rrows.size());
    for (size_t r = 0; r < rrows.size(); r++) s.rsell.h_tile[r] = s.h_node_tile[rrows[r]];
    sell_build_halo(s, s.rsell);
  }
  s.rsell.slice_layer = ar.alloc<int32_t>(s.rsell.n_slices);
  if (s.rsell.n_slices) {
    k_slice_layer<<<nb(s.rsell.n_slices), 256, 0, st>>>(s.rsell.rows, s.rsell.n_rows, s.rsell.n_slices, s.rsell.L,
                                                        s.layer, s.rsell.slice_layer);
    MTS_LAUNCH_CHECK();
  }

  // colour classes: constraints closer than 2R + 2 delta get different colours,
  // so the responses (support radius R) of one class never overlap.  This is a
  // scheduling choice; every entry of H is still the single-load response.
  const double sep = 2.0 * Rr + 2.0 * s.prm.delta;
  const double own = Rr + 0.5 * s.prm.delta;
  std::vector<int32_t> color(s.nc, -1);
  {
    const double cs = sep;
    double lo[3] = {0, 0, 0};
    for (int a = 0; a < dim; a++) lo[a] = s.p.pd_lo[a] - 2 * s.prm.delta;
    auto key = [&](int64_t q, int64_t off[3]) {
      int64_t c[3] = {0, 0, 0};
      for (int a = 0; a < dim; a++) c[a] = (int64_t)std::floor((s.pos[(int64_t)s.h_cn[q] * dim + a] - lo[a]) / cs) + off[a];
      return (c[2] * 1000003LL + c[1]) * 1000003LL + c[0];
    };
    std::unordered_map<int64_t, std::vector<int32_t>> cells;
    int64_t zero[3] = {0, 0, 0};
    for (int64_t q = 0; q < s.nc; q++) cells[key(q, zero)].push_back((int32_t)q);
    auto d2 = [&](int64_t a, int64_t b) {
      double r = 0;
      for (int c = 0; c < dim; c++) {
        double t = s.pos[(int64_t)s.h_cn[a] * dim + c] - s.pos[(int64_t)s.h_cn[b] * dim + c];
        r += t * t;
      }
      return r;
    };
    std::vector<char> used;
    int zr = dim == 3 ? 1 : 0;
    for (int64_t q = 0; q < s.nc; q++) {
      used.assign(used.size(), 0);
      for (int dz = -zr; dz <= zr; dz++)
        for (int dy = -1; dy <= 1; dy++)
          for (int dxx = -1; dxx <= 1; dxx++) {
            int64_t off[3] = {dxx, dy, dz};
            auto it = cells.find(key(q, off));
            if (it == cells.end()) continue;
            for (int32_t p : it->second)
              if (color[p] >= 0 && d2(p, q) <= sep * sep) {
                if ((int64_t)used.size() <= color[p]) used.resize(color[p] + 1, 0);
                used[color[p]] = 1;
              }
          }
      int c = 0;
      while (c < (int)used.size() && used[c]) c++;
      color[q] = c;
    }
    s.n_colors = 0;
    for (int32_t c : color) s.n_colors = std::max<int64_t>(s.n_colors, c + 1);
    // owner[c][q]: the constraint of colour c whose support can reach q
    std::vector<int32_t> owner((size_t)(s.n_colors * s.nc), -1);
    for (int64_t q = 0; q < s.nc; q++)
      for (int dz = -zr; dz <= zr; dz++)
        for (int dy = -1; dy <= 1; dy++)
          for (int dxx = -1; dxx <= 1; dxx++) {
            int64_t off[3] = {dxx, dy, dz};
            auto it = cells.find(key(q, off));
            if (it == cells.end()) continue;
            for (int32_t p : it->second)
              if (d2(p, q) <= own * own) owner[(size_t)color[p] * s.nc + q] = p;
          }
    int32_t *dcolor = ar.alloc<int32_t>(s.nc);
    int32_t *downer = ar.alloc<int32_t>(owner.size());
    MTS_HIP(hipMemcpyAsync(dcolor, color.data(), sizeof(int32_t) * s.nc, hipMemcpyHostToDevice, st));
    MTS_HIP(hipMemcpyAsync(downer, owner.data(), sizeof(int32_t) * owner.size(), hipMemcpyHostToDevice, st));
    s.ccolor = dcolor;
    s.owner = downer;
    MTS_HIP(hipStreamSynchronize(st));
  }
  s.nrhs = dim == 2 ? 8 : 6;
  {
    // loaded constraint nodes of every batch of unit loads (colours bt * cpb ..)
    const int cpb = s.nrhs / dim;
    const int64_t nbatch = (s.n_colors + cpb - 1) / cpb;
    std::vector<int32_t> boff(nbatch + 1, 0), bnodes;
    std::vector<std::vector<int32_t>> members(s.n_colors);
    for (int64_t q = 0; q < s.nc; q++) members[color[q]].push_back(s.h_cn[q]);
    for (int64_t bt = 0; bt < nbatch; bt++) {
      for (int64_t c = bt * cpb; c < std::min<int64_t>((bt + 1) * cpb, s.n_colors); c++)
        bnodes.insert(bnodes.end(), members[c].begin(), members[c].end());
      boff[bt + 1] = (int32_t)bnodes.size();
    }
    s.h_batch_off = boff;
    // constraints by cell of the response reach, to find those near a changed bond
    s.h_ccolor = color;
    s.own_r = own;
    s.h_ccells.clear();
    for (int64_t q = 0; q < s.nc; q++) {
      int64_t c[3] = {0, 0, 0};
      for (int a = 0; a < dim; a++) c[a] = (int64_t)std::floor(s.pos[(int64_t)s.h_cn[q] * dim + a] / own);
      s.h_ccells[(c[2] * 1000003LL + c[1]) * 1000003LL + c[0]].push_back((int32_t)q);
    }
    s.built_mask = ar.alloc<uint64_t>(std::max<int64_t>(s.sell.n_words, 1));
    s.dirty = ar.alloc<uint8_t>(N);
    s.ccolor_sub = ar.alloc<int32_t>(std::max<int64_t>(s.nc, 1));
    s.csel = ar.alloc<uint8_t>(std::max<int64_t>(s.nc, 1));
    s.built_valid = false;
    s.batch_nodes = ar.alloc<int32_t>(std::max<size_t>(bnodes.size(), 1));
    if (!bnodes.empty())
      MTS_HIP(hipMemcpyAsync(s.batch_nodes, bnodes.data(), sizeof(int32_t) * bnodes.size(), hipMemcpyHostToDevice, st));
    s.batch_layer = ar.alloc<int32_t>(std::max<int64_t>(s.rsell.n_slices, 1));
    MTS_HIP(hipStreamSynchronize(st));
  }
  size_t wsz = (size_t)s.nrhs * dim * N;
  s.Wu[0] = ar.alloc<double>(wsz);
  s.Wu[1] = ar.alloc<double>(wsz);
  s.Wv = ar.alloc<double>(wsz);
  s.Wa = ar.alloc<double>(wsz);
  // responses stay exact zeros outside the link region (rows there are read
  // as neighbours and never written)
  for (double *q : {s.Wu[0], s.Wu[1], s.Wv, s.Wa}) MTS_HIP(hipMemsetAsync(q, 0, sizeof(double) * wsz, st));
  for (int q = 0; q < s.build_streams - 1; q++) {
    Solver::BuildSet &B = s.bset[q];
    B.u[0] = ar.alloc<double>(wsz);
    B.u[1] = ar.alloc<double>(wsz);
    B.v = ar.alloc<double>(wsz);
    B.a = ar.alloc<double>(wsz);
    B.layer = ar.alloc<int32_t>(std::max<int64_t>(s.rsell.n_slices, 1));
    for (double *q : {B.u[0], B.u[1], B.v, B.a}) MTS_HIP(hipMemsetAsync(q, 0, sizeof(double) * wsz, st));
  }
  if (!s.bfork && s.build_streams > 1) {
    MTS_HIP(hipEventCreateWithFlags(&s.bfork, hipEventDisableTiming));
    for (int q = 0; q < s.build_streams - 1; q++) {
      MTS_HIP(hipStreamCreateWithFlags(&s.bstream[q], hipStreamNonBlocking));  // default priority
      MTS_HIP(hipEventCreateWithFlags(&s.bjoin[q], hipEventDisableTiming));
    }
  }
  for (int k = 0; k < 2; k++) s.Wxu[k] = ar.alloc<double>((size_t)2 * dim * N);
  link_records_init(s);
  s.lam = ar.alloc<double>(s.nl);
  s.lam0 = ar.alloc<double>(s.nl);
  s.rhs = ar.alloc<double>(s.nl);
  MTS_HIP(hipMemsetAsync(s.lam, 0, sizeof(double) * s.nl, st));
  MTS_HIP(hipMemsetAsync(s.lam0, 0, sizeof(double) * s.nl, st));
  s.H = ar.alloc<double>((size_t)s.nl * s.nl);
  s.keep_h = s.nl <= 4096;
  // connected components of the coupling graph: constraints farther apart than
  // both the response reach and two element diagonals never share an entry of H
  {
    const double h = s.p.fe_h;
    const double J = std::max(Rr, 2.0 * std::sqrt((double)dim) * h) + s.prm.delta;
    std::vector<int32_t> parent(s.nc);
    for (int64_t q = 0; q < s.nc; q++) parent[q] = (int32_t)q;
    auto find = [&](int32_t a) {
      while (parent[a] != a) a = parent[a] = parent[parent[a]];
      return a;
    };
    double lo[3] = {0, 0, 0};
    for (int a = 0; a < dim; a++) lo[a] = s.p.pd_lo[a] - 2 * s.prm.delta;
    auto key = [&](int64_t q, const int64_t off[3]) {
      int64_t c[3] = {0, 0, 0};
      for (int a = 0; a < dim; a++) c[a] = (int64_t)std::floor((s.pos[(int64_t)s.h_cn[q] * dim + a] - lo[a]) / J) + off[a];
      return (c[2] * 1000003LL + c[1]) * 1000003LL + c[0];
    };
    std::unordered_map<int64_t, std::vector<int32_t>> cells;
    const int64_t zero[3] = {0, 0, 0};
    for (int64_t q = 0; q < s.nc; q++) cells[key(q, zero)].push_back((int32_t)q);
    int zr = dim == 3 ? 1 : 0;
    for (int64_t q = 0; q < s.nc; q++)
      for (int dz = -zr; dz <= zr; dz++)
        for (int dy = -1; dy <= 1; dy++)
          for (int dxx = -1; dxx <= 1; dxx++) {
            const int64_t off[3] = {dxx, dy, dz};
            auto it = cells.find(key(q, off));
            if (it == cells.end()) continue;
            for (int32_t p : it->second) {
              double r2 = 0;
              for (int a = 0; a < dim; a++) {
                double t = s.pos[(int64_t)s.h_cn[p] * dim + a] - s.pos[(int64_t)s.h_cn[q] * dim + a];
                r2 += t * t;
              }
              if (r2 <= J * J) {
                int32_t ra = find((int32_t)q), rb = find(p);
                if (ra != rb) parent[std::max(ra, rb)] = std::min(ra, rb);
              }
            }
          }
    if (s.fe_beta > 0.0)  // A^-1 of the implicit FE step couples every constraint
      for (int64_t q = 0; q < s.nc; q++) parent[q] = 0;
    std::vector<int32_t> label(s.nc, -1);
    std::vector<std::vector<int32_t>> comps;
    for (int64_t q = 0; q < s.nc; q++) {
      int32_t r = find((int32_t)q);
      if (label[r] < 0) {
        label[r] = (int32_t)comps.size();
        comps.emplace_back();
      }
      for (int d = 0; d < dim; d++) comps[label[r]].push_back((int32_t)(q * dim + d));
    }
    sym_blocks_setup(s, comps);
    vlog(s, "coupling: %lld constraints, %lld colours, %lld components, largest %lld dofs", (long long)s.nc,
         (long long)s.n_colors, (long long)s.sym.n_comp, (long long)s.sym.n_max);
  }
  for (int k = 0; k < 2; k++) {
    s.mask_snap[k] = ar.alloc<uint64_t>(s.sell.n_words);
    MTS_HIP(hipEventCreateWithFlags(&s.flag_event[k], hipEventDisableTiming));
  }
  if (s.fe_beta > 0.0) {
    fe_implicit_hf(s);  // does not change when bonds break
    vlog(s, "fe: implicit block of H done");
  }
  coupling_rebuild(s, s.sell.mask);
}

// Unit-load responses on the given bond states (full-lattice layout), H, and its inverse.
// After the first build a rebuild recomputes only the columns of the
// constraints whose response reach holds a node with a bond changed since the
// last build: every other column would come out bit for bit the same (its
// link run sees the same bond states, and the loads of one colour never reach
// a common node), so H, and its inverse, equal those of a full rebuild.
void coupling_rebuild(Solver &s, const uint64_t *full_mask) {
  const int dim = s.dim;
  hipStream_t st = s.stream;
  const int64_t nl = s.nl;
  sell_regather_mask(s, s.rsell, full_mask);
  const int cpb = s.nrhs / dim;  // colours per batch
  const bool first = !s.built_valid;
  bool all = first || !s.incremental;
  std::vector<int32_t> sel;  // constraints to recompute when not all
  if (!all) {
    MTS_HIP(hipMemsetAsync(s.dirty, 0, (size_t)s.N, st));
    if (s.sell.n_slices) {
      k_dirty_nodes<<<(unsigned)s.sell.n_slices, WAVE, 0, st>>>(s.sell.word_off, s.sell.n_slices, s.sell.rows,
                                                                s.sell.n_rows, s.sell.L, s.built_mask, full_mask,
                                                                s.dirty);
      MTS_LAUNCH_CHECK();
    }
    std::vector<uint8_t> dirty((size_t)s.N);
    MTS_HIP(hipMemcpyAsync(dirty.data(), s.dirty, (size_t)s.N, hipMemcpyDeviceToHost, st));
    MTS_HIP(hipStreamSynchronize(st));
    std::vector<uint8_t> mark((size_t)s.nc, 0);
    const double r2max = s.own_r * s.own_r;
    const int zr = dim == 3 ? 1 : 0;
    for (int64_t i = 0; i < s.N; i++) {
      if (!dirty[i]) continue;
      const double *xi = &s.pos[(size_t)i * dim];
      int64_t c[3] = {0, 0, 0};
      for (int a = 0; a < dim; a++) c[a] = (int64_t)std::floor(xi[a] / s.own_r);
      for (int dz = -zr; dz <= zr; dz++)
        for (int dy = -1; dy <= 1; dy++)
          for (int dxx = -1; dxx <= 1; dxx++) {
            auto it = s.h_ccells.find(((c[2] + dz) * 1000003LL + (c[1] + dy)) * 1000003LL + (c[0] + dxx));
            if (it == s.h_ccells.end()) continue;
            for (int32_t q : it->second) {
              if (mark[q]) continue;
              double r2 = 0.0;
              for (int a = 0; a < dim; a++) {
                const double t = s.pos[(size_t)s.h_cn[q] * dim + a] - xi[a];
                r2 += t * t;
              }
              if (r2 <= r2max) mark[q] = 1;
            }
          }
    }
    for (int64_t q = 0; q < s.nc; q++)
      if (mark[q]) sel.push_back((int32_t)q);
    if ((int64_t)sel.size() == s.nc) all = true;
  }
  // batches of cpb colours: their RHS (colour, direction) and loaded PD nodes
  std::vector<int32_t> bcol, boff{0}, bnodes;
  if (all) {
    for (int64_t c = 0; c < s.n_colors; c++) bcol.push_back((int32_t)c);
  } else {
    std::map<int32_t, std::vector<int32_t>> members;  // colour -> loaded PD nodes
    for (int32_t q : sel) members[s.h_ccolor[q]].push_back(s.h_cn[q]);
    for (auto &kv : members) bcol.push_back(kv.first);
    int64_t k = 0;
    for (auto &kv : members) {
      bnodes.insert(bnodes.end(), kv.second.begin(), kv.second.end());
      if (++k % cpb == 0 || k == (int64_t)members.size()) boff.push_back((int32_t)bnodes.size());
    }
  }
  const int64_t nbatch = ((int64_t)bcol.size() + cpb - 1) / cpb;
  std::vector<int32_t> rcd((size_t)std::max<int64_t>(nbatch, 1) * 32, -1);
  for (int64_t bt = 0; bt < nbatch; bt++)
    for (int b = 0; b < s.nrhs; b++) {
      const int64_t c = bt * cpb + b / dim;
      rcd[bt * 32 + b] = c < (int64_t)bcol.size() ? bcol[c] : -1;
      rcd[bt * 32 + 16 + b] = b % dim;
    }
  int32_t *drcd = s.arena.alloc<int32_t>(rcd.size());
  MTS_HIP(hipMemcpyAsync(drcd, rcd.data(), sizeof(int32_t) * rcd.size(), hipMemcpyHostToDevice, st));
  int32_t *dnodes = nullptr;
  const int32_t *load_color = s.ccolor;
  const uint8_t *csel = nullptr;
  // host sources of the copies below stay alive until the stream is synchronised
  std::vector<int32_t> sub;
  std::vector<uint8_t> cs;
  if (all) {
    MTS_HIP(hipMemsetAsync(s.H, 0, sizeof(double) * nl * nl, st));
  } else {
    sub.assign((size_t)s.nc, -1);
    cs.assign((size_t)s.nc, 0);
    for (int32_t q : sel) {
      sub[q] = s.h_ccolor[q];
      cs[q] = 1;
    }
    MTS_HIP(hipMemcpyAsync(s.ccolor_sub, sub.data(), sizeof(int32_t) * s.nc, hipMemcpyHostToDevice, st));
    MTS_HIP(hipMemcpyAsync(s.csel, cs.data(), (size_t)s.nc, hipMemcpyHostToDevice, st));
    dnodes = s.arena.alloc<int32_t>(std::max<size_t>(bnodes.size(), 1));
    if (!bnodes.empty())
      MTS_HIP(hipMemcpyAsync(dnodes, bnodes.data(), sizeof(int32_t) * bnodes.size(), hipMemcpyHostToDevice, st));
    load_color = s.ccolor_sub;
    csel = s.csel;
    k_zero_cols<<<nb(nl * nl), 256, 0, st>>>(nl, dim, csel, s.H);
    MTS_LAUNCH_CHECK();
  }
  // the batches are independent: each has its own right-hand sides, writes
  // only its own constraints' columns of H, and runs on stream bt mod nst
  // (the solver's build streams) with that stream's buffers, forked from and
  // joined into st
  const int nst = (int)std::min<int64_t>(s.build_streams, std::max<int64_t>(nbatch, 1));
  if (nst > 1) {
    MTS_HIP(hipEventRecord(s.bfork, st));
    for (int q = 0; q < nst - 1; q++) MTS_HIP(hipStreamWaitEvent(s.bstream[q], s.bfork, 0));
  }
  struct StreamBack {  // s.stream is the launch stream of link_substep
    Solver &s;
    hipStream_t st;
    ~StreamBack() { s.stream = st; }
  } back{s, st};
  for (int64_t bt = 0; bt < nbatch; bt++) {
    const int q = (int)(bt % nst);
    hipStream_t sq = q ? s.bstream[q - 1] : st;
    double *const u0 = q ? s.bset[q - 1].u[0] : s.Wu[0], *const u1 = q ? s.bset[q - 1].u[1] : s.Wu[1];
    double *const wv = q ? s.bset[q - 1].v : s.Wv, *const wa = q ? s.bset[q - 1].a : s.Wa;
    int32_t *const layer = q ? s.bset[q - 1].layer : s.batch_layer;
    const int32_t *rc = &rcd[bt * 32], *rd = &rcd[bt * 32 + 16];
    if (s.rsell.n_slices) {
      const int32_t *bn = all ? s.batch_nodes + s.h_batch_off[bt] : dnodes + boff[bt];
      const int32_t nbn = all ? s.h_batch_off[bt + 1] - s.h_batch_off[bt] : boff[bt + 1] - boff[bt];
      k_batch_layer<<<(unsigned)s.rsell.n_slices, WAVE, 0, sq>>>(s.x, s.N, dim, s.rsell.rows, s.rsell.n_rows,
                                                                 s.rsell.n_slices, s.rsell.L, bn, nbn, s.prm.delta,
                                                                 s.m, layer);
      MTS_LAUNCH_CHECK();
    }
    s.stream = sq;
    int k = 0;  // substep 1 starts every response from rest, so no clearing is needed
    const double *uk[2] = {u0, u1};
    double *uw[2] = {u0, u1};
    for (int j = 1; j <= s.m; j++) {
      link_substep(s, j, uk[k], uw[k ^ 1], wv, wa, load_color, rc, rd, s.nrhs, layer);
      k ^= 1;
    }
    s.stream = st;
    k_extract<<<nb(s.nc), 256, 0, sq>>>(s.nc, dim, nl, s.nrhs, s.cn, s.owner, drcd + bt * 32, drcd + bt * 32 + 16,
                                        wv, csel, s.H);
    MTS_LAUNCH_CHECK();
  }
  if (nst > 1)
    for (int q = 0; q < nst - 1; q++) {
      MTS_HIP(hipEventRecord(s.bjoin[q], s.bstream[q]));
      MTS_HIP(hipStreamWaitEvent(st, s.bjoin[q], 0));
    }
  if (s.fe_beta > 0.0) {
    k_add_dense<<<nb(nl * nl), 256, 0, st>>>(nl * nl, nl, dim, csel, s.fe_HF, s.H);
  } else {
    dim3 blk(16, 16), grd((unsigned)((s.nc + 15) / 16), (unsigned)((s.nc + 15) / 16));
    k_add_hf<<<grd, blk, 0, st>>>(s.nc, dim, s.nen, nl, s.cel, s.conn, s.cw, s.mF, s.bc, s.prm.hdtF, s.p.fe_n[0],
                                  s.p.fe_n[1], csel, s.H);
  }
  MTS_LAUNCH_CHECK();
  MTS_HIP(hipMemcpyAsync(s.built_mask, full_mask, sizeof(uint64_t) * s.sell.n_words, hipMemcpyDeviceToDevice, st));
  MTS_HIP(hipStreamSynchronize(st));  // before the host tables go away
  s.arena.release(drcd);
  if (dnodes) s.arena.release(dnodes);
  s.built_valid = true;
  const int64_t ncols = all ? s.nc : (int64_t)sel.size();
  if (!first) s.n_rebuild_cols += ncols;
  vlog(s, "coupling: unit-load responses of %lld of %lld constraints done (%lld colour batches)", (long long)ncols,
       (long long)s.nc, (long long)nbatch);
  if (s.keep_h) {
    if (!s.Hcopy) s.Hcopy = s.arena.alloc<double>((size_t)nl * nl);
    MTS_HIP(hipMemcpyAsync(s.Hcopy, s.H, sizeof(double) * nl * nl, hipMemcpyDeviceToDevice, st));
  }
  sym_blocks_build(s);
  MTS_HIP(hipStreamSynchronize(st));
  vlog(s, "coupling: H inverted");
}

void coupling_free(Solver &s) {
  for (int q = 0; q < Solver::kBuildStreams - 1; q++) {
    if (s.bstream[q]) {
      (void)hipStreamSynchronize(s.bstream[q]);
      (void)hipStreamDestroy(s.bstream[q]);
    }
    if (s.bjoin[q]) (void)hipEventDestroy(s.bjoin[q]);
    s.bstream[q] = nullptr;
    s.bjoin[q] = nullptr;
  }
  if (s.bfork) (void)hipEventDestroy(s.bfork);
  s.bfork = nullptr;
}

bool coupling_solve_and_correct(Solver &s, bool fuse_next_fe, int snap_slot) {
  coupling_lambda(s);
  if (s.fe_beta > 0.0) fe_implicit_correct(s);  // a full-mesh solve, not a ring pass
  return coupling_link(s, fuse_next_fe && s.fe_beta == 0.0, snap_slot);
}

void coupling_lambda(Solver &s) {
  hipStream_t st = s.stream;
  hipEvent_t e0 = nullptr;
  s.prof_begin(MTS_KT_LAMBDA, &e0);
  k_rhs<<<nb(s.nc), 256, 0, st>>>(s.nc, s.dim, s.nen, s.cn, s.cel, s.conn, s.cw, s.vt, s.v, s.N, s.rhs, s.sym.rpos,
                                  s.sym.rperm);
  MTS_LAUNCH_CHECK();
  sym_blocks_apply(s, s.rhs, s.sym.rperm, s.lam, s.lam0);  // lambda_0 <- lambda_m for the next macro step too
  s.prof_end(MTS_KT_LAMBDA, e0);
}

bool coupling_link(Solver &s, bool fuse_next_fe, int snap_slot) {
  // FE: the ring nodes' final update; PD: U = V + Y lambda_m by re-running the
  // link problem with lambda_m.  Both need only lambda_m, so the FE pass runs as
  // extra workgroups of the first link launch; with fuse_next_fe (2D, m >= 3)
  // the next macro step's FE free step (element forces, then the gather)
  // follows in the second and third (they read the FE state this step's
  // correction leaves).
  const bool ring = s.n_ring && s.fe_beta == 0.0;  // the implicit correction ran before
  if (!s.rsell.n_rows) {
    if (ring) fe_correct(s);
    if (snap_slot >= 0) snapshot_masks(s, snap_slot);
    return false;
  }
  const bool fuse = fuse_next_fe && s.m >= 3 && s.dim == 2;
  hipEvent_t e1 = nullptr;
  s.prof_begin(MTS_KT_LINK, &e1);
  // m substeps from rest; the last one adds W_m into the PD state directly
  int k = 0;
  bool snapped = snap_slot < 0;
  for (int j = 1; j <= s.m; j++) {
    int side = kSideNone;
    if (j == 1 && ring) side = kSideRing;
    if (fuse && j == 2) side = kSideElem;
    if (fuse && j == 3) side = kSideGather;
    if (side == kSideNone && !snapped) {  // the first launch with room saves the bond states
      side = kSideSnap;
      snapped = true;
    }
    link_final_substep(s, j, k, j == s.m, side, snap_slot);
    k ^= 1;
  }
  if (!snapped) snapshot_masks(s, snap_slot);
  s.prof_end(MTS_KT_LINK, e1);
  return fuse;
}

}  // namespace mts
