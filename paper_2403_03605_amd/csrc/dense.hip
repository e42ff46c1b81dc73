// Dense FP64 linear algebra for the multiplier system of Eq. 49: each diagonal
// block of the symmetric positive-definite matrix H (one per connected
// component of the coupling graph) is inverted once per (re)build by blocked
// in-place Gauss-Jordan elimination (no pivoting, SPD) and stored as its
// lower-triangle 64 x 64 tiles; every macro step applies the inverse with a
// tile-parallel symmetric GEMV whose partial sums are combined in a fixed order.
#include "internal.h"

#include <algorithm>
#include <cmath>

namespace mts {

namespace {

constexpr int NB = 64;

// Invert the kb x kb pivot block A[k0:k0+kb, k0:k0+kb] in LDS (Gauss-Jordan),
// padded to 64 x 64 with the identity (whose inverse is itself).  Thread t
// owns column t % 64 and rows 16 (t / 64) .. 16 (t / 64) + 15.
__global__ __launch_bounds__(256) void k_pivot_inverse(const double *A, int64_t n, int64_t k0, int kb,
                                                      double *pinv) {
  __shared__ double M[NB][NB + 1];
  __shared__ double rowp[NB], colp[NB];
  const int c = threadIdx.x & 63, r0 = (threadIdx.x >> 6) * 16;
  for (int q = 0; q < 16; q++) {
    const int r = r0 + q;
    M[r][c] = (r < kb && c < kb) ? A[(k0 + r) * n + k0 + c] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int p = 0; p < NB; p++) {
    const double d = 1.0 / M[p][p];
    if (threadIdx.x < NB) {
      rowp[c] = (c == p) ? d : M[p][c] * d;
      colp[c] = M[c][p];
    }
    __syncthreads();
    for (int q = 0; q < 16; q++) {
      const int r = r0 + q;
      double v;
      if (r == p) v = rowp[c];
      else if (c == p) v = -colp[r] * d;
      else v = M[r][c] - colp[r] * rowp[c];
      M[r][c] = v;
    }
    __syncthreads();
  }
  for (int q = 0; q < 16; q++) {
    const int r = r0 + q;
    if (r < kb && c < kb) pinv[r * kb + c] = M[r][c];
  }
}

// C[i][t] = A[i][k0+t] (0 on the pivot rows);  R[t][j] = (Pinv A[K,:])[t][j], R[:,K] = Pinv.
__global__ void k_panels(const double *A, int64_t n, int64_t k0, int kb, const double *pinv, double *C,
                         double *R) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = n * kb;
  if (idx >= total) return;
  // C part: idx -> (i, t)
  {
    int64_t i = idx / kb;
    int t = (int)(idx % kb);
    bool inK = i >= k0 && i < k0 + kb;
    C[i * kb + t] = inK ? 0.0 : A[i * n + k0 + t];
  }
  // R part: idx -> (t, j)
  {
    int t = (int)(idx / n);
    int64_t j = idx % n;
    double r;
    if (j >= k0 && j < k0 + kb) {
      r = pinv[t * kb + (j - k0)];
    } else {
      r = 0.0;
      for (int s = 0; s < kb; s++) r += pinv[t * kb + s] * A[(k0 + s) * n + j];
    }
    R[(int64_t)t * n + j] = r;
  }
}

__global__ void k_write_panels(double *A, int64_t n, int64_t k0, int kb, const double *R) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * kb) return;
  {
    int t = (int)(idx / n);
    int64_t j = idx % n;
    A[(k0 + t) * n + j] = R[(int64_t)t * n + j];
  }
  {
    int64_t i = idx / kb;
    int t = (int)(idx % kb);
    if (!(i >= k0 && i < k0 + kb)) A[i * n + k0 + t] = 0.0;
  }
}

// A -= C R over the whole matrix: a rank-kb update, kb <= 64, on the FP64
// matrix cores.  64 x 64 output tile per workgroup; wave w owns rows
// [16 w, 16 w + 16) of the tile as four 16 x 16 MFMA tiles, accumulating onto
// the loaded A with the negated C operand.  Operand layout of
// v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// accumulator register g of lane l is row 4 g + l / 16, column l % 16.
__global__ __launch_bounds__(256) void k_rank_update(double *A, int64_t n, int kb, const double *C,
                                                     const double *R) {
  __shared__ double Cs[NB][NB + 1];
  __shared__ double Rs[NB][NB + 1];
  const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
  for (int t = threadIdx.x; t < 64 * NB; t += 256) {
    const int r = t / NB, c = t % NB;
    const int64_t i = i0 + r;
    Cs[r][c] = (i < n && c < kb) ? -C[i * kb + c] : 0.0;
    const int64_t j = j0 + c;
    Rs[r][c] = (r < kb && j < n) ? R[(int64_t)r * n + j] : 0.0;
  }
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  typedef double d4 __attribute__((ext_vector_type(4)));
  d4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; t++)
#pragma unroll
    for (int g = 0; g < 4; g++) {
      const int64_t i = i0 + 16 * w + 4 * g + lk, j = j0 + 16 * t + lr;
      acc[t][g] = (i < n && j < n) ? A[i * n + j] : 0.0;
    }
  __syncthreads();
  for (int k0 = 0; k0 < NB; k0 += 4) {
    const double a = Cs[16 * w + lr][k0 + lk];
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const double b = Rs[k0 + lk][16 * t + lr];
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; t++)
#pragma unroll
    for (int g = 0; g < 4; g++) {
      const int64_t i = i0 + 16 * w + 4 * g + lk, j = j0 + 16 * t + lr;
      if (i < n && j < n) A[i * n + j] = acc[t][g];
    }
}

}  // namespace

void dense_spd_inverse(Solver &s, double *A, int64_t n) {
  hipStream_t st = s.stream;
  if (n <= 0) return;
  if (!s.tmpA) {  // sized for the largest block this solver will ever invert
    const int64_t cap = std::max<int64_t>(n, s.sym.n_max);
    s.tmpA = s.arena.alloc<double>((size_t)cap * NB);
    s.tmpB = s.arena.alloc<double>((size_t)cap * NB);
    s.pinv = s.arena.alloc<double>((size_t)NB * NB);
  }
  for (int64_t k0 = 0; k0 < n; k0 += NB) {
    int kb = (int)std::min<int64_t>(NB, n - k0);
    k_pivot_inverse<<<1, 256, 0, st>>>(A, n, k0, kb, s.pinv);
    MTS_LAUNCH_CHECK();
    int64_t tot = n * kb;
    k_panels<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(A, n, k0, kb, s.pinv, s.tmpA, s.tmpB);
    MTS_LAUNCH_CHECK();
    k_write_panels<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(A, n, k0, kb, s.tmpB);
    MTS_LAUNCH_CHECK();
    dim3 grid((unsigned)((n + 63) / 64), (unsigned)((n + 63) / 64));
    k_rank_update<<<grid, 256, 0, st>>>(A, n, kb, s.tmpA, s.tmpB);
    MTS_LAUNCH_CHECK();
  }
}


// ---------------------------------------------------------------------------
// Block-diagonal inverse in packed lower-triangle tiles
// ---------------------------------------------------------------------------
namespace {

constexpr int TS = 64;  // tile side

// work[i][j] = H[idx[i]][idx[j]] for one component
__global__ void k_gather_block(const double *H, int64_t nl, const int32_t *idx, int64_t n, double *work) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  int64_t i = t / n, j = t % n;
  work[t] = H[(int64_t)idx[i] * nl + idx[j]];
}

// packed[tile (I, J), J <= I][r][c] = work[64 I + r][64 J + c] (0 outside)
__global__ void k_pack_tiles(const double *work, int64_t n, int64_t T, double *packed) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t ntile = T * (T + 1) / 2;
  if (t >= ntile * TS * TS) return;
  int64_t tile = t / (TS * TS);
  int e = (int)(t % (TS * TS));
  int64_t I = (int64_t)((sqrt(8.0 * (double)tile + 1.0) - 1.0) / 2.0);
  while (I * (I + 1) / 2 > tile) I--;
  while ((I + 1) * (I + 2) / 2 <= tile) I++;
  int64_t J = tile - I * (I + 1) / 2;
  int64_t i = I * TS + e / TS, j = J * TS + e % TS;
  packed[t] = (i < n && j < n) ? work[i * n + j] : 0.0;
}

// One workgroup per tile: row partial A_IJ x_J (for block row I) and, off the
// diagonal, column partial A_IJ^T x_I (for block row J).  Four threads share a
// row (or column), 16 products each, combined by a fixed butterfly.
__global__ __launch_bounds__(256) void k_sym_tiles(const double *packed, const int32_t *tile_meta,
                                                   const int64_t *off, const int32_t *idx, const double *r,
                                                   double *rowpart, double *colpart) {
  __shared__ double A[TS][TS + 1];
  __shared__ double xI[TS], xJ[TS];
  const int64_t tile = blockIdx.x;
  const int comp = tile_meta[tile * 3 + 0], I = tile_meta[tile * 3 + 1], J = tile_meta[tile * 3 + 2];
  const int64_t base = off[comp], n = off[comp + 1] - off[comp];
  const double2 *src = reinterpret_cast<const double2 *>(packed + tile * TS * TS);
  const int t = threadIdx.x;
  double2 v[8];
#pragma unroll
  for (int q = 0; q < 8; q++) v[q] = src[q * 256 + t];
  if (t < TS) {
    int64_t gi = (int64_t)I * TS + t, gj = (int64_t)J * TS + t;
    xI[t] = gi < n ? r[idx[base + gi]] : 0.0;
    xJ[t] = gj < n ? r[idx[base + gj]] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 8; q++) {
    const int e = 2 * (q * 256 + t);
    A[e / TS][e % TS] = v[q].x;
    A[e / TS][e % TS + 1] = v[q].y;
  }
  __syncthreads();
  const int line = t >> 2, part = t & 3;
  double rs = 0.0, cs = 0.0;
#pragma unroll
  for (int k = 0; k < 16; k++) {
    rs += A[line][part * 16 + k] * xJ[part * 16 + k];
    cs += A[part * 16 + k][line] * xI[part * 16 + k];
  }
  rs += __shfl_xor(rs, 1, WAVE);
  rs += __shfl_xor(rs, 2, WAVE);
  cs += __shfl_xor(cs, 1, WAVE);
  cs += __shfl_xor(cs, 2, WAVE);
  if (part == 0) {
    rowpart[tile * TS + line] = rs;
    if (I != J) colpart[tile * TS + line] = cs;
  }
}

// y[idx[i]] = sum_{J <= I} rowpart(I, J) + sum_{J > I} colpart(J, I).  One
// workgroup per block row; wave w takes every 4th contribution and the four
// wave sums are added in a fixed order.
__global__ __launch_bounds__(256) void k_sym_reduce(const int64_t *off, const int64_t *tile_base,
                                                    const int32_t *row_comp, const int32_t *row_block,
                                                    const int32_t *idx, const double *rowpart,
                                                    const double *colpart, double *y) {
  __shared__ double part[4][TS];
  const int64_t c = row_comp[blockIdx.x], I = row_block[blockIdx.x];
  const int64_t n = off[c + 1] - off[c], T = (n + TS - 1) / TS, tb = tile_base[c];
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
  double s = 0.0;
  for (int64_t k = w; k < T; k += 4) {
    s += k <= I ? rowpart[(tb + I * (I + 1) / 2 + k) * TS + lane] : colpart[(tb + k * (k + 1) / 2 + I) * TS + lane];
  }
  part[w][lane] = s;
  __syncthreads();
  if (w == 0) {
    const int64_t i = I * TS + lane;
    const double tot = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
    if (i < n) y[idx[off[c] + i]] = tot;
  }
}

}  // namespace

void sym_blocks_setup(Solver &s, const std::vector<std::vector<int32_t>> &comps) {
  auto &B = s.sym;
  DeviceArena &ar = s.arena;
  hipStream_t st = s.stream;
  B.n_comp = (int64_t)comps.size();
  B.h_off.assign(B.n_comp + 1, 0);
  B.h_idx.clear();
  std::vector<int64_t> tbase(B.n_comp + 1, 0);
  std::vector<int32_t> meta;
  B.n_max = 0;
  for (int64_t c = 0; c < B.n_comp; c++) {
    int64_t n = (int64_t)comps[c].size();
    B.h_off[c + 1] = B.h_off[c] + n;
    B.h_idx.insert(B.h_idx.end(), comps[c].begin(), comps[c].end());
    B.n_max = std::max(B.n_max, n);
    int64_t T = (n + TS - 1) / TS;
    tbase[c + 1] = tbase[c] + T * (T + 1) / 2;
    for (int64_t I = 0; I < T; I++)
      for (int64_t J = 0; J <= I; J++) {
        meta.push_back((int32_t)c);
        meta.push_back((int32_t)I);
        meta.push_back((int32_t)J);
      }
  }
  B.n_tiles = tbase[B.n_comp];
  B.idx = ar.alloc<int32_t>(B.h_idx.size());
  B.off = ar.alloc<int64_t>(B.n_comp + 1);
  B.tile_meta = ar.alloc<int32_t>(meta.size());
  B.tile_base = ar.alloc<int64_t>(B.n_comp + 1);
  B.packed = ar.alloc<double>((size_t)B.n_tiles * TS * TS);
  B.rowpart = ar.alloc<double>((size_t)B.n_tiles * TS);
  B.colpart = ar.alloc<double>((size_t)B.n_tiles * TS);
  B.work = ar.alloc<double>((size_t)B.n_max * B.n_max);
  std::vector<int32_t> rc, rb;
  for (int64_t c = 0; c < B.n_comp; c++) {
    int64_t T = (B.h_off[c + 1] - B.h_off[c] + TS - 1) / TS;
    for (int64_t I = 0; I < T; I++) {
      rc.push_back((int32_t)c);
      rb.push_back((int32_t)I);
    }
  }
  B.n_rows = (int64_t)rc.size();
  B.row_comp = ar.alloc<int32_t>(rc.size());
  B.row_block = ar.alloc<int32_t>(rb.size());
  MTS_HIP(hipMemcpyAsync(B.row_comp, rc.data(), sizeof(int32_t) * rc.size(), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemcpyAsync(B.row_block, rb.data(), sizeof(int32_t) * rb.size(), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemcpyAsync(B.idx, B.h_idx.data(), sizeof(int32_t) * B.h_idx.size(), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemcpyAsync(B.off, B.h_off.data(), sizeof(int64_t) * (B.n_comp + 1), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemcpyAsync(B.tile_meta, meta.data(), sizeof(int32_t) * meta.size(), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemcpyAsync(B.tile_base, tbase.data(), sizeof(int64_t) * (B.n_comp + 1), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemsetAsync(B.colpart, 0, sizeof(double) * B.n_tiles * TS, st));
  MTS_HIP(hipStreamSynchronize(st));
}

// Invert every component block of H (already assembled in s.H) and pack it.
void sym_blocks_build(Solver &s) {
  auto &B = s.sym;
  hipStream_t st = s.stream;
  std::vector<int64_t> tbase(B.n_comp + 1, 0);
  for (int64_t c = 0; c < B.n_comp; c++) {
    int64_t n = B.h_off[c + 1] - B.h_off[c];
    int64_t T = (n + TS - 1) / TS;
    tbase[c + 1] = tbase[c] + T * (T + 1) / 2;
    k_gather_block<<<(unsigned)((n * n + 255) / 256), 256, 0, st>>>(s.H, s.nl, B.idx + B.h_off[c], n, B.work);
    MTS_LAUNCH_CHECK();
    dense_spd_inverse(s, B.work, n);
    int64_t ne = T * (T + 1) / 2 * TS * TS;
    k_pack_tiles<<<(unsigned)((ne + 255) / 256), 256, 0, st>>>(B.work, n, T, B.packed + tbase[c] * TS * TS);
    MTS_LAUNCH_CHECK();
    vlog(s, "coupling: block %lld of %lld inverted (%lld dofs)", (long long)(c + 1), (long long)B.n_comp,
         (long long)n);
  }
}

void sym_blocks_apply(Solver &s, const double *r, double *y) {
  auto &B = s.sym;
  if (!B.n_tiles) return;
  k_sym_tiles<<<(unsigned)B.n_tiles, 256, 0, s.stream>>>(B.packed, B.tile_meta, B.off, B.idx, r, B.rowpart,
                                                         B.colpart);
  MTS_LAUNCH_CHECK();
  k_sym_reduce<<<(unsigned)B.n_rows, 256, 0, s.stream>>>(B.off, B.tile_base, B.row_comp, B.row_block, B.idx,
                                                        B.rowpart, B.colpart, y);
  MTS_LAUNCH_CHECK();
}

}  // namespace mts
