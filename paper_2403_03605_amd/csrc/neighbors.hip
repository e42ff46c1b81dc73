// Neighbour families H_delta(x_i) = {k != i : |x_k - x_i| <= delta} (Sec. 2.1),
// built on the device with a cell list, stored as canonical CSR (rows ascending)
// (re-laid as sliced ELL for the bond pass in layout.hip).
#include "internal.h"

#include <algorithm>

namespace mts {

namespace {

constexpr int kThreads = 256;

inline unsigned blocks_for(int64_t n, int t = kThreads) { return (unsigned)((n + t - 1) / t); }

// ---------------------------------------------------------------- scan
__global__ void scan_block_i64(const int64_t *in, int64_t *out, int64_t *block_sums, int64_t n) {
  __shared__ int64_t sh[1024];
  int64_t base = (int64_t)blockIdx.x * 1024;
  int t = threadIdx.x;  // 256 threads, 4 items each
  int64_t v[4];
  int64_t s = 0;
  for (int q = 0; q < 4; q++) {
    int64_t idx = base + t * 4 + q;
    v[q] = idx < n ? in[idx] : 0;
    s += v[q];
  }
  sh[t] = s;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int64_t add = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  int64_t run = sh[t] - s;  // exclusive prefix of this thread
  for (int q = 0; q < 4; q++) {
    int64_t idx = base + t * 4 + q;
    if (idx < n) out[idx] = run;
    run += v[q];
  }
  if (t == 255 && block_sums) block_sums[blockIdx.x] = sh[255];
}

__global__ void scan_add_i64(int64_t *out, const int64_t *offs, int64_t n) {
  int64_t idx = (int64_t)blockIdx.x * 1024 + threadIdx.x * 4;
  int64_t o = offs[blockIdx.x];
  for (int q = 0; q < 4; q++)
    if (idx + q < n) out[idx + q] += o;
}

// ---------------------------------------------------------------- cell list
struct Grid {
  double lo[3];
  double cs;
  int64_t nc[3];
};

__device__ inline int64_t cell_coord(double x, double lo, double cs, int64_t nc) {
  int64_t c = (int64_t)floor((x - lo) / cs);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__global__ void k_cell_of(const double *x, int64_t N, int dim, Grid g, int32_t *cell, int32_t *count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int64_t c0 = cell_coord(x[i], g.lo[0], g.cs, g.nc[0]);
  int64_t c1 = cell_coord(x[N + i], g.lo[1], g.cs, g.nc[1]);
  int64_t c2 = dim == 3 ? cell_coord(x[2 * N + i], g.lo[2], g.cs, g.nc[2]) : 0;
  int64_t c = (c2 * g.nc[1] + c1) * g.nc[0] + c0;
  cell[i] = (int32_t)c;
  atomicAdd(&count[c], 1);
}

__global__ void k_i32_to_i64(const int32_t *a, int64_t *b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

__global__ void k_scatter_cells(const int32_t *cell, int64_t N, const int64_t *start, int32_t *fill,
                                int32_t *items) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int c = cell[i];
  int slot = atomicAdd(&fill[c], 1);
  items[start[c] + slot] = (int32_t)i;
}

// |x_k - x_i|^2 evaluated as ((dx*dx + dy*dy) + dz*dz), contraction off.
__device__ inline double dist2_soa(const double *x, int64_t N, int dim, int64_t i, int64_t k) {
  double d0 = x[k] - x[i];
  double d1 = x[N + k] - x[N + i];
  double r2 = d0 * d0 + d1 * d1;
  if (dim == 3) {
    double d2 = x[2 * N + k] - x[2 * N + i];
    r2 = r2 + d2 * d2;
  }
  return r2;
}

template <bool kFill>
__global__ void k_family(const double *x, int64_t N, int dim, Grid g, const int32_t *cell,
                         const int64_t *cstart, const int32_t *items, double d2, int64_t *rowlen,
                         const int64_t *rp, int32_t *col) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int64_t c = cell[i];
  int64_t cx = c % g.nc[0], cy = (c / g.nc[0]) % g.nc[1], cz = c / (g.nc[0] * g.nc[1]);
  int64_t cnt = 0;
  int64_t out = kFill ? rp[i] : 0;
  int zr = dim == 3 ? 1 : 0;
  for (int dz = -zr; dz <= zr; dz++)
    for (int dy = -1; dy <= 1; dy++)
      for (int dx = -1; dx <= 1; dx++) {
        int64_t ax = cx + dx, ay = cy + dy, az = cz + dz;
        if (ax < 0 || ay < 0 || az < 0 || ax >= g.nc[0] || ay >= g.nc[1] || az >= g.nc[2]) continue;
        int64_t q = (az * g.nc[1] + ay) * g.nc[0] + ax;
        for (int64_t t = cstart[q]; t < cstart[q + 1]; t++) {
          int64_t k = items[t];
          if (k == i) continue;
          if (dist2_soa(x, N, dim, i, k) <= d2) {
            if (kFill) col[out + cnt] = (int32_t)k;
            cnt++;
          }
        }
      }
  if (!kFill) {
    rowlen[i] = cnt;
  } else {
    // canonical order: ascending neighbour id (insertion sort of a short row)
    int32_t *r = col + out;
    for (int64_t a = 1; a < cnt; a++) {
      int32_t key = r[a];
      int64_t b = a - 1;
      while (b >= 0 && r[b] > key) {
        r[b + 1] = r[b];
        b--;
      }
      r[b + 1] = key;
    }
  }
}

__global__ void k_i64_to_i32(const int64_t *a, int32_t *b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (int32_t)a[i];
}

}  // namespace

void exclusive_scan_i64(hipStream_t st, DeviceArena &ar, const int64_t *in, int64_t *out, int64_t n) {
  if (n <= 0) return;
  int64_t nb = (n + 1023) / 1024;
  if (nb == 1) {
    scan_block_i64<<<1, 256, 0, st>>>(in, out, nullptr, n);
    MTS_LAUNCH_CHECK();
    return;
  }
  int64_t *sums = ar.alloc<int64_t>(nb);
  int64_t *offs = ar.alloc<int64_t>(nb);
  scan_block_i64<<<(unsigned)nb, 256, 0, st>>>(in, out, sums, n);
  MTS_LAUNCH_CHECK();
  exclusive_scan_i64(st, ar, sums, offs, nb);
  scan_add_i64<<<(unsigned)nb, 256, 0, st>>>(out, offs, n);
  MTS_LAUNCH_CHECK();
  MTS_HIP(hipStreamSynchronize(st));
  ar.release(sums);
  ar.release(offs);
}

void build_neighbors(Solver &s) {
  const int dim = s.dim;
  const int64_t N = s.N;
  hipStream_t st = s.stream;
  DeviceArena &ar = s.arena;
  // Cell list with cells of side delta: two points within delta fall in the
  // same or adjacent cells, so 3^dim cells are searched per node.
  Grid g{};
  g.cs = s.prm.delta;
  for (int a = 0; a < 3; a++) {
    g.lo[a] = 0.0;
    g.nc[a] = 1;
  }
  for (int a = 0; a < dim; a++) {
    double lo = s.pos[a], hi = s.pos[a];
    for (int64_t i = 0; i < N; i++) {
      lo = std::min(lo, s.pos[i * dim + a]);
      hi = std::max(hi, s.pos[i * dim + a]);
    }
    g.lo[a] = lo;
    g.nc[a] = (int64_t)std::floor((hi - lo) / g.cs) + 1;
  }
  int64_t ncell = g.nc[0] * g.nc[1] * g.nc[2];
  if (ncell > (int64_t)1 << 30) throw ArgError{"cell grid too large"};
  int32_t *cell = ar.alloc<int32_t>(N);
  int32_t *count = ar.alloc<int32_t>(ncell);
  int32_t *fill = ar.alloc<int32_t>(ncell);
  int64_t *count64 = ar.alloc<int64_t>(ncell + 1);
  int64_t *cstart = ar.alloc<int64_t>(ncell + 1);
  int32_t *items = ar.alloc<int32_t>(N);
  MTS_HIP(hipMemsetAsync(count, 0, sizeof(int32_t) * ncell, st));
  MTS_HIP(hipMemsetAsync(fill, 0, sizeof(int32_t) * ncell, st));
  MTS_HIP(hipMemsetAsync(count64, 0, sizeof(int64_t) * (ncell + 1), st));
  k_cell_of<<<blocks_for(N), kThreads, 0, st>>>(s.x, N, dim, g, cell, count);
  MTS_LAUNCH_CHECK();
  k_i32_to_i64<<<blocks_for(ncell), kThreads, 0, st>>>(count, count64, ncell);
  MTS_LAUNCH_CHECK();
  exclusive_scan_i64(st, ar, count64, cstart, ncell + 1);
  k_scatter_cells<<<blocks_for(N), kThreads, 0, st>>>(cell, N, cstart, fill, items);
  MTS_LAUNCH_CHECK();

  int64_t *rowlen = ar.alloc<int64_t>(N + 1);
  int64_t *rp64 = ar.alloc<int64_t>(N + 1);
  MTS_HIP(hipMemsetAsync(rowlen, 0, sizeof(int64_t) * (N + 1), st));
  k_family<false><<<blocks_for(N), kThreads, 0, st>>>(s.x, N, dim, g, cell, cstart, items, s.prm.d2,
                                                       rowlen, nullptr, nullptr);
  MTS_LAUNCH_CHECK();
  exclusive_scan_i64(st, ar, rowlen, rp64, N + 1);
  int64_t nnz = 0;
  MTS_HIP(hipMemcpyAsync(&nnz, rp64 + N, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MTS_HIP(hipStreamSynchronize(st));
  if (nnz >= ((int64_t)1 << 31)) throw ArgError{"more than 2^31 bonds"};
  s.nnz = nnz;
  s.rp = ar.alloc<int32_t>(N + 1);
  s.csr_col = ar.alloc<int32_t>(nnz);
  k_i64_to_i32<<<blocks_for(N + 1), kThreads, 0, st>>>(rp64, s.rp, N + 1);
  MTS_LAUNCH_CHECK();
  k_family<true><<<blocks_for(N), kThreads, 0, st>>>(s.x, N, dim, g, cell, cstart, items, s.prm.d2, nullptr,
                                                      rp64, s.csr_col);
  MTS_LAUNCH_CHECK();
  MTS_HIP(hipStreamSynchronize(st));
  for (void *q : {(void *)cell, (void *)count, (void *)fill, (void *)count64, (void *)cstart,
                  (void *)items, (void *)rowlen, (void *)rp64})
    ar.release(q);

  // Rows of the bond layout in spatial tile order (32 x 8 nodes in 2D, 32 x 16
  // with eight-wavefront workgroups; 8 x 4 x 4 or 4 x 4 x 4 in 3D; ascending id
  // inside a tile): a workgroup's rows and their neighbours then form a compact
  // patch, which keeps the neighbour gathers of consecutive workgroups in the
  // same L2 and the staged neighbour lists short.
  if (s.halo_waves == 0) s.halo_waves = (dim == 3 && s.precision == MTS_MIXED) ? 8 : 4;
  std::vector<int32_t> rows(N);
  for (int64_t i = 0; i < N; i++) rows[i] = (int32_t)i;
  if (s.tiled != 0 && s.p.dx > 0.0) {
    double lo[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < dim; a++) {
      lo[a] = s.pos[a];
      for (int64_t i = 0; i < N; i++) lo[a] = std::min(lo[a], s.pos[(size_t)i * dim + a]);
    }
    // 3D tiles of 16 x halo_waves nodes: one workgroup at 4 lanes per row
    const double ext2[3] = {32.0, s.halo_waves == 8 ? 16.0 : 8.0, 1.0}, ext3[3] = {s.halo_waves == 8 ? 8.0 : 4.0, 4.0, 4.0};
    const double *ext = dim == 2 ? ext2 : ext3;
    std::vector<int64_t> key(N);
    int64_t nt[3] = {1, 1, 1};
    std::vector<int64_t> tc((size_t)N * 3);
    for (int64_t i = 0; i < N; i++)
      for (int a = 0; a < dim; a++) {
        const int64_t t = (int64_t)std::floor((s.pos[(size_t)i * dim + a] - lo[a]) / (ext[a] * s.p.dx));
        tc[(size_t)i * 3 + a] = std::max<int64_t>(t, 0);
        nt[a] = std::max(nt[a], tc[(size_t)i * 3 + a] + 1);
      }
    for (int64_t i = 0; i < N; i++)
      key[i] = (tc[(size_t)i * 3 + 2] * nt[1] + tc[(size_t)i * 3 + 1]) * nt[0] + tc[(size_t)i * 3 + 0];
    std::stable_sort(rows.begin(), rows.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    s.sell.h_tile.resize(N);
    for (int64_t r = 0; r < N; r++) s.sell.h_tile[r] = key[rows[r]];
    s.h_node_tile = key;
    std::vector<int32_t> row_of(N);
    for (int64_t r = 0; r < N; r++) row_of[rows[r]] = (int32_t)r;
    s.sell.row_of = ar.alloc<int32_t>(N);
    MTS_HIP(hipMemcpyAsync(s.sell.row_of, row_of.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, st));
    MTS_HIP(hipStreamSynchronize(st));
  }
  // In 3D a workgroup at 4 lanes per row covers one tile, whose staged
  // neighbour records fit LDS.
  int L = s.force_lanes ? s.force_lanes : pick_lanes(N, dim);
  if (!s.force_lanes && dim == 3 && s.halo && s.tiled != 0) L = std::max(L, 4);
  build_sell(s, s.sell, rows, nullptr, L);
  s.sell.wg_waves = s.halo_waves;
  // the bond pass addresses its arrays with 32-bit byte offsets
  const uint64_t lim = (uint64_t)1 << 32;
  if ((uint64_t)(s.sell.n_slots + (int64_t)kSpareIters * WAVE) * 8 >= lim || (uint64_t)N * 2 * dim * 8 >= lim)
    throw ArgError{"problem too large for one solver (bond or node arrays beyond 4 GiB)"};
}

}  // namespace mts
