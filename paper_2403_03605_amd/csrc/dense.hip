// Dense FP64 linear algebra for the multiplier system of Eq. 49: each diagonal
// block of the symmetric positive-definite matrix H (one per connected
// component of the coupling graph) is inverted once per (re)build and stored
// as its lower-triangle 64 x 64 tiles; every macro step applies the inverse
// with a tile-parallel symmetric GEMV whose partial sums are combined in a
// fixed order.
//
// Inversion: the symmetric sweep operator, directly on the packed lower tiles.
// Sweeping pivot block K of a symmetric A with P = A_KK^-1:
//   A_IJ <- A_IJ - A_IK P A_KJ   (I, J not in K),
//   A_IK <- A_IK P,  A_KJ <- P A_KJ,  A_KK <- -P,
// keeps A symmetric, so only the lower tiles are touched; sweeping every block
// leaves -A^-1.  Sweeping a block equals sweeping its parts one after another,
// so the pivot blocks are four tiles (256) wide: the diagonal block is swept
// tile by tile on its own ten tiles (which leaves -P there), and then one
// rank-256 update on the FP64 matrix cores passes over the whole matrix -- a
// quarter of the memory traffic of 64-wide pivots for the same flops.
#include "internal.h"

#include <algorithm>
#include <cmath>

namespace mts {

namespace {

constexpr int TS = 64;  // tile side
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline int64_t tile_row(int64_t tile) {
  int64_t I = (int64_t)((sqrt(8.0 * (double)tile + 1.0) - 1.0) / 2.0);
  while (I * (I + 1) / 2 > tile) I--;
  while ((I + 1) * (I + 2) / 2 <= tile) I++;
  return I;
}

__device__ inline int64_t tile_index(int64_t I, int64_t J) { return I * (I + 1) / 2 + J; }

// packed[tile (I, J), J <= I][r][c] = H[idx[64 I + r]][idx[64 J + c]] (0 outside)
__global__ void k_pack_lower(const double *H, int64_t nl, const int32_t *idx, int64_t n, int64_t T, double *packed) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T * (T + 1) / 2 * TS * TS) return;
  const int64_t tile = t / (TS * TS);
  const int e = (int)(t % (TS * TS));
  const int64_t I = tile_row(tile), J = tile - I * (I + 1) / 2;
  const int64_t i = I * TS + e / TS, j = J * TS + e % TS;
  packed[t] = (i < n && j < n) ? H[(int64_t)idx[i] * nl + idx[j]] : 0.0;
}

// P = inverse of the diagonal tile (k, k) (symmetric part), its rows/columns
// past n padded with the identity.  The tile is swept in LDS in four 16-wide
// sub-pivots (the same sweep operator as the whole matrix, which leaves -A^-1):
// wavefront 0 inverts the 16 x 16 pivot block by Gauss-Jordan in registers
// (no pivoting: every pivot block is a Schur complement of an SPD tile, hence
// SPD), exchanging the pivot row and column with shuffles; then all four
// wavefronts form the panel W = V B^-1 and update the tile, rank 16.
__global__ __launch_bounds__(256) void k_tile_inverse(const double *packed, int64_t k, int64_t n, double *P) {
  constexpr int SB = 16;  // sub-pivot width
  __shared__ double M[TS][TS + 1];
  __shared__ double Vs[TS][SB + 1], Ws[TS][SB + 1], Bi[SB][SB + 1];
  const int t = threadIdx.x;
  const double *D = packed + tile_index(k, k) * TS * TS;
  const int kb = (int)std::min<int64_t>(TS, n - k * TS);
  for (int e = t; e < TS * TS; e += blockDim.x) {
    const int r = e / TS, c = e % TS;
    M[r][c] = (r < kb && c < kb) ? D[e] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  const int r0 = (t >> 4) * 4, c0 = (t & 15) * 4;  // this thread's 4 x 4 block of the tile
  for (int o = 0; o < TS; o += SB) {
    if (t < WAVE) {
      // lane t holds B[br][bc .. bc + 3] of the pivot block B = M[o.., o..]
      const int br = t >> 2, bc = (t & 3) * 4;
      double b[4];
#pragma unroll
      for (int j = 0; j < 4; j++) b[j] = M[o + br][o + bc + j];
#pragma unroll
      for (int p = 0; p < SB; p++) {
        double rp[4];  // pivot row p, columns bc .. bc + 3
#pragma unroll
        for (int j = 0; j < 4; j++) rp[j] = __shfl(b[j], 4 * p + (t & 3), WAVE);
        const double cp = __shfl(b[p & 3], 4 * br + (p >> 2), WAVE);   // B[br][p]
        const double piv = __shfl(b[p & 3], 4 * p + (p >> 2), WAVE);  // B[p][p]
        const double d = 1.0 / piv;
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int c = bc + j;
          if (br == p) b[j] = (c == p) ? d : rp[j] * d;
          else if (c == p) b[j] = -cp * d;
          else b[j] = b[j] - cp * (rp[j] * d);
        }
      }
#pragma unroll
      for (int j = 0; j < 4; j++) Bi[br][bc + j] = b[j];
    }
    for (int e = t; e < TS * SB; e += blockDim.x) Vs[e / SB][e % SB] = M[e / SB][o + e % SB];
    __syncthreads();
    {
      // panel W = V B^-1 (64 x 16), one 16 x 16 output tile per wavefront
      const int lane = t & (WAVE - 1), w = t >> 6;
      const int lr = lane & 15, lk = lane >> 4;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k4 = 0; k4 < SB; k4 += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[16 * w + lr][k4 + lk], Bi[k4 + lk][lr], acc, 0, 0, 0);
#pragma unroll
      for (int g = 0; g < 4; g++) Ws[16 * w + 4 * g + lk][lr] = acc[g];
    }
    __syncthreads();
    // rank-16 update A_IJ - A_IK P A_KJ = M - V W^T on the matrix cores: each
    // lane owns the 16 entries of the 16 x 16 output layout (rows 16 w + 4 g + lk,
    // columns 16 t + lr), so the update is in place
    {
      const int lane = t & (WAVE - 1), w = t >> 6;
      const int lr = lane & 15, lk = lane >> 4;
      d4 acc[4];
#pragma unroll
      for (int tt = 0; tt < 4; tt++)
#pragma unroll
        for (int g = 0; g < 4; g++) acc[tt][g] = M[16 * w + 4 * g + lk][16 * tt + lr];
#pragma unroll
      for (int k4 = 0; k4 < SB; k4 += 4) {
        const double a = -Vs[16 * w + lr][k4 + lk];
#pragma unroll
        for (int tt = 0; tt < 4; tt++)
          acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Ws[16 * tt + lr][k4 + lk], acc[tt], 0, 0, 0);
      }
#pragma unroll
      for (int tt = 0; tt < 4; tt++)
#pragma unroll
        for (int g = 0; g < 4; g++) {
          const int r = 16 * w + 4 * g + lk, c = 16 * tt + lr;
          const bool rin = r >= o && r < o + SB, cin = c >= o && c < o + SB;
          double v = acc[tt][g];
          if (rin && cin) v = -Bi[r - o][c - o];  // A_KK <- -P
          else if (cin) v = Ws[r][c - o];         // A_IK <- A_IK P
          else if (rin) v = Ws[c][r - o];         // A_KJ <- P A_KJ = (A_JK P)^T
          M[r][c] = v;
        }
    }
    __syncthreads();
  }
  // the sweep left -A^-1; P is its negated symmetric part (symmetric P keeps
  // the sweep of the whole matrix exactly symmetric, as its storage assumes)
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int bb = 0; bb < 4; bb++) {
      const int r = r0 + a, c = c0 + bb;
      P[r * TS + c] = -0.5 * (M[r][c] + M[c][r]);
    }
}

// Load a 64 x 64 tile (row-major source, optionally transposed) into LDS.
__device__ inline void load_tile(double (*dst)[TS + 1], const double *src, bool transpose) {
  for (int e = threadIdx.x; e < TS * TS; e += blockDim.x) {
    const int r = e / TS, c = e % TS;
    if (transpose) dst[c][r] = src[e];
    else dst[r][c] = src[e];
  }
}

// acc (wave w's 16 rows, 4 column tiles) += sign * X[16 w .., :] * Y where
// Y[kk][col] = Ycol(col, kk) (ycol_major) or Y[kk][col] (row-major).
template <bool YT>
__device__ inline void mfma_rows(d4 acc[4], const double (*X)[TS + 1], const double (*Y)[TS + 1], double sign) {
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  for (int k0 = 0; k0 < TS; k0 += 4) {
    const double a = sign * X[16 * w + lr][k0 + lk];
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const double b = YT ? Y[16 * t + lr][k0 + lk] : Y[k0 + lk][16 * t + lr];
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
    }
  }
}

// Panel of pivot tile k: V_I = A_Ik (from tile (I, k) or the transpose of
// tile (k, I)) and W_I = V_I P, one workgroup per tile row I = r0 + block.
__global__ __launch_bounds__(256) void k_sweep_panel(const double *packed, int64_t k, const double *P, double *V,
                                                    double *W, int64_t r0) {
  __shared__ double Vs[TS][TS + 1], Ps[TS][TS + 1];
  const int64_t I = r0 + blockIdx.x;
  const bool below = I >= k;
  load_tile(Vs, packed + (below ? tile_index(I, k) : tile_index(k, I)) * TS * TS, !below);
  load_tile(Ps, P, false);
  __syncthreads();
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  d4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; t++) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  mfma_rows<false>(acc, Vs, Ps, 1.0);
  double *Vo = V + I * TS * TS, *Wo = W + I * TS * TS;
#pragma unroll
  for (int t = 0; t < 4; t++)
#pragma unroll
    for (int g = 0; g < 4; g++) {
      const int r = 16 * w + 4 * g + lk, c = 16 * t + lr;
      Wo[r * TS + c] = acc[t][g];
      Vo[r * TS + c] = Vs[r][c];
    }
}

// Sweep of pivot tile k over the lower tiles of the diagonal block that starts
// at tile k0 (one workgroup per tile; tile index local to that block).
// Interior tiles: A_IJ -= W_I V_J^T on the matrix cores with the operands read
// straight from the (cache-resident) panels: lane group lk of a wavefront
// supplies the reduction indices 16 lk .. 16 lk + 15 (a permutation of the
// 64-term sums, so each lane reads contiguous 128-byte runs), no LDS.
__global__ __launch_bounds__(256) void k_sweep_update(double *packed, int64_t k, const double *P, const double *V,
                                                     const double *W, int64_t k0) {
  const int64_t li = tile_row(blockIdx.x);
  const int64_t I = k0 + li, J = k0 + (int64_t)blockIdx.x - li * (li + 1) / 2;
  double *A = packed + tile_index(I, J) * TS * TS;
  if (I == k || J == k) {
    // pivot row / column / diagonal: -P, W_I, or W_J^T
    const double *src = (I == k && J == k) ? P : (J == k ? W + I * TS * TS : W + J * TS * TS);
    const double sg = (I == k && J == k) ? -1.0 : 1.0;
    const bool tr = I == k && J != k;
    for (int e = threadIdx.x; e < TS * TS; e += blockDim.x) {
      const int r = e / TS, c = e % TS;
      A[e] = sg * (tr ? src[c * TS + r] : src[e]);
    }
    return;
  }
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  d4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; t++)
#pragma unroll
    for (int g = 0; g < 4; g++) acc[t][g] = A[(16 * w + 4 * g + lk) * TS + 16 * t + lr];
  const double2 *wrow = reinterpret_cast<const double2 *>(W + I * TS * TS + (16 * w + lr) * TS + 16 * lk);
  double a[16];
#pragma unroll
  for (int q = 0; q < 8; q++) {
    const double2 v = wrow[q];
    a[2 * q] = -v.x;
    a[2 * q + 1] = -v.y;
  }
  // two halves of the 16 reduction steps; inside a half the four accumulator
  // chains are interleaved so consecutive MFMAs are independent
#pragma unroll
  for (int hh = 0; hh < 2; hh++) {
    double b[4][8];
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const double2 *vrow =
          reinterpret_cast<const double2 *>(V + J * TS * TS + (16 * t + lr) * TS + 16 * lk + 8 * hh);
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const double2 v = vrow[q];
        b[t][2 * q] = v.x;
        b[t][2 * q + 1] = v.y;
      }
    }
#pragma unroll
    for (int s2 = 0; s2 < 8; s2++)
#pragma unroll
      for (int t = 0; t < 4; t++)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[8 * hh + s2], b[t][s2], acc[t], 0, 0, 0);
  }
#pragma unroll
  for (int t = 0; t < 4; t++)
#pragma unroll
    for (int g = 0; g < 4; g++) A[(16 * w + 4 * g + lk) * TS + 16 * t + lr] = acc[t][g];
}

// Dense 256 x 256 (row stride KB) multiplier block of the current pivot block:
// Pb = -(swept diagonal block) = A_KK^-1, both triangles from the lower tiles.
constexpr int NB = 4;         // tiles per pivot block
constexpr int KB = NB * TS;   // pivot block width
__global__ void k_pblock(const double *packed, int64_t k0, int nb, double *Pb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int K = nb * TS;
  if (e >= K * K) return;
  const int r = e / K, c = e % K;
  const int hi = r > c ? r : c, lo = r > c ? c : r;
  const double *t = packed + tile_index(k0 + hi / TS, k0 + lo / TS) * TS * TS;
  Pb[r * KB + c] = -t[(hi % TS) * TS + lo % TS];
}

// Panel of pivot block K = tiles k0 .. k0 + nb - 1 for tile row I (not in K):
// V_I = A_IK (64 x 64 nb, row stride KB) and the column tile c of W_I = V_I Pb.
// Grid (T, nb): workgroup (I, c) accumulates over the nb tiles of K on MFMA.
__global__ __launch_bounds__(256) void k_block_panel(const double *packed, int64_t k0, int nb, const double *Pb,
                                                    double *V, double *W) {
  __shared__ double Vs[TS][TS + 1], Ps[TS][TS + 1];
  const int64_t I = blockIdx.x;
  const int c = blockIdx.y;
  if (I >= k0 && I < k0 + nb) return;  // uniform per workgroup
  d4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; t++) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  for (int kk = 0; kk < nb; kk++) {
    const int64_t k = k0 + kk;
    const bool below = I > k;
    __syncthreads();  // the previous step's tiles are no longer read
    load_tile(Vs, packed + (below ? tile_index(I, k) : tile_index(k, I)) * TS * TS, !below);
    for (int e = threadIdx.x; e < TS * TS; e += blockDim.x) Ps[e / TS][e % TS] = Pb[(kk * TS + e / TS) * KB + c * TS + e % TS];
    __syncthreads();
    mfma_rows<false>(acc, Vs, Ps, 1.0);
    if (kk == c)  // V_I's column tile c
      for (int e = threadIdx.x; e < TS * TS; e += blockDim.x) V[(I * TS + e / TS) * KB + c * TS + e % TS] = Vs[e / TS][e % TS];
  }
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int t = 0; t < 4; t++)
#pragma unroll
    for (int g = 0; g < 4; g++) W[(I * TS + 16 * w + 4 * g + lk) * KB + c * TS + 16 * t + lr] = acc[t][g];
}

// Sweep of pivot block K = tiles k0 .. k0 + nb - 1 over every lower tile:
//   I, J not in K: A_IJ -= W_I V_J^T (rank 64 nb, on MFMA);
//   J in K:        A_IJ <- column tile of W_I;
//   I in K:        A_IJ <- transpose of a column tile of W_J;
//   I, J in K:     unchanged (the diagonal sweep left -P there).
__global__ __launch_bounds__(256, 4) void k_block_update(double *packed, int64_t k0, int nb, const double *V,
                                                     const double *W) {
  const int64_t tile = blockIdx.x;
  const int64_t I = tile_row(tile), J = tile - I * (I + 1) / 2;
  const int64_t k1 = k0 + nb;
  const bool iin = I >= k0 && I < k1, jin = J >= k0 && J < k1;
  if (iin && jin) return;
  double *A = packed + tile * TS * TS;
  if (iin || jin) {
    // J in K (then I >= k1): W_I's column tile J - k0; I in K (then J < k0): W_J's column tile I - k0, transposed
    const double *src = jin ? W + I * TS * KB + (J - k0) * TS : W + J * TS * KB + (I - k0) * TS;
    for (int e = threadIdx.x; e < TS * TS; e += blockDim.x) {
      const int r = e / TS, c = e % TS;
      A[e] = jin ? src[r * KB + c] : src[c * KB + r];
    }
    return;
  }
  // V_J's 64-column chunks pass through LDS once per workgroup (all four
  // wavefronts need all of V_J); each wavefront reads its own 16 rows of W_I.
  __shared__ double Vs[TS][TS + 2];  // row stride keeps 16-byte alignment
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  d4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; t++)
#pragma unroll
    for (int g = 0; g < 4; g++) acc[t][g] = A[(16 * w + 4 * g + lk) * TS + 16 * t + lr];
#pragma unroll 1
  for (int kk = 0; kk < nb; kk++) {
    if (kk) __syncthreads();  // the previous chunk is no longer read
    {
      const int r = threadIdx.x >> 2, c0 = (threadIdx.x & 3) * 16;
      const double2 *src = reinterpret_cast<const double2 *>(V + (J * TS + r) * KB + kk * TS + c0);
#pragma unroll
      for (int q = 0; q < 8; q++) *reinterpret_cast<double2 *>(&Vs[r][c0 + 2 * q]) = src[q];
    }
    const double2 *wrow = reinterpret_cast<const double2 *>(W + (I * TS + 16 * w + lr) * KB + kk * TS + 16 * lk);
    double a[16];
#pragma unroll
    for (int q = 0; q < 8; q++) {
      const double2 v = wrow[q];
      a[2 * q] = -v.x;
      a[2 * q + 1] = -v.y;
    }
    __syncthreads();
#pragma unroll
    for (int hh = 0; hh < 2; hh++) {
      double b[4][8];
#pragma unroll
      for (int t = 0; t < 4; t++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const double2 v = *reinterpret_cast<const double2 *>(&Vs[16 * t + lr][16 * lk + 8 * hh + 2 * q]);
          b[t][2 * q] = v.x;
          b[t][2 * q + 1] = v.y;
        }
#pragma unroll
      for (int s2 = 0; s2 < 8; s2++)
#pragma unroll
        for (int t = 0; t < 4; t++)
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[8 * hh + s2], b[t][s2], acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; t++)
#pragma unroll
    for (int g = 0; g < 4; g++) A[(16 * w + 4 * g + lk) * TS + 16 * t + lr] = acc[t][g];
}

__global__ void k_negate(double *a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = -a[i];
}

// Row partial A_IJ x_J (for block row I) and, off the diagonal, column
// partial A_IJ^T x_I (for block row J) of every packed tile, one wavefront per
// tile, from registers (no workgroup barrier).  Load q of lane l brings
// entries (2q + h, c0) and (2q + h, c0 + 1), h = l / 32, c0 = 2 (l % 32); the
// tile is taken in quarters of 8 loads.  Column sums accumulate in the
// lane and pair up across h; each row's 32 two-entry products are summed over
// its half-wavefront by recursive halving (a fixed order: deterministic).
__device__ __forceinline__ double pick(bool hi, double a, double b) { return hi ? b : a; }

// Largest |entry| of every packed tile (one wavefront per tile).
__global__ void k_tile_absmax(const double *packed, int64_t n_tiles, double *out) {
  const int64_t tile = blockIdx.x;
  const int lane = threadIdx.x;
  if (tile >= n_tiles) return;
  const double *src = packed + tile * TS * TS;
  double m = 0.0;
  for (int q = lane; q < TS * TS; q += WAVE) m = fmax(m, fabs(src[q]));
  for (int off = WAVE / 2; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off, WAVE));
  if (lane == 0) out[tile] = m;
}

// Listed tiles rewritten in FP32 (round to nearest) into the first half of
// their own slot: one workgroup per tile reads the whole tile before writing.
__global__ __launch_bounds__(256) void k_tiles_to_f32(double *packed, const int32_t *tiles) {
  double v[TS * TS / 256];
  double *tp = packed + (int64_t)tiles[blockIdx.x] * TS * TS;
#pragma unroll
  for (int q = 0; q < TS * TS / 256; q++) v[q] = tp[q * 256 + threadIdx.x];
  __syncthreads();
  float *dst = reinterpret_cast<float *>(tp);
#pragma unroll
  for (int q = 0; q < TS * TS / 256; q++) dst[q * 256 + threadIdx.x] = (float)v[q];
}

// Eight 16-byte pieces of a tile for this lane: pairs of entries (row 2 q + h,
// columns c0, c0 + 1), from the FP64 tile or from its FP32 copy in the first
// half of the same slot (converted exactly to FP64).
__device__ __forceinline__ void load_pairs(const double *tile, bool f32, int q0, int lane, double2 e[8]) {
  if (f32) {
    const float2 *src = reinterpret_cast<const float2 *>(tile);
#pragma unroll
    for (int q = 0; q < 8; q++) {
      const float2 v = src[(q0 + q) * WAVE + lane];
      e[q] = double2{(double)v.x, (double)v.y};
    }
  } else {
    const double2 *src = reinterpret_cast<const double2 *>(tile);
#pragma unroll
    for (int q = 0; q < 8; q++) e[q] = src[(q0 + q) * WAVE + lane];
  }
}

// Row sums of quarter qt of a tile (rows 16 qt .. 16 qt + 15): p[q] holds
// this lane's two-entry products of row 2 (8 qt + q) + h; recursive halving
// over the 32 lanes of the half-wavefront, then one lane in four writes.
__device__ __forceinline__ void sym_quarter_rows(const double p[8], int lane, int qt, double *row_tile) {
  const int h = lane >> 5;
  const bool b4 = (lane >> 4) & 1, b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1;
  double p4[4], p2[2];
#pragma unroll
  for (int kk = 0; kk < 4; kk++) p4[kk] = pick(b4, p[kk], p[4 + kk]) + __shfl_xor(pick(b4, p[4 + kk], p[kk]), 16, WAVE);
#pragma unroll
  for (int kk = 0; kk < 2; kk++) p2[kk] = pick(b3, p4[kk], p4[2 + kk]) + __shfl_xor(pick(b3, p4[2 + kk], p4[kk]), 8, WAVE);
  double p1 = pick(b2, p2[0], p2[1]) + __shfl_xor(pick(b2, p2[1], p2[0]), 4, WAVE);
  p1 += __shfl_xor(p1, 2, WAVE);
  p1 += __shfl_xor(p1, 1, WAVE);
  // the four lanes 4k .. 4k + 3 of the half hold row 2 (8 qt + k) + h, k = (lane % 32) / 4
  if ((lane & 3) == 0) row_tile[2 * (8 * qt + ((lane & 31) >> 2)) + h] = p1;
}

// A kept tile's header, made wave-uniform, and this lane's x_I and x_J
// entries (r in component-block order, zero-padded), staged in LDS.
struct SymTile {
  int64_t tile;
  bool f32, offd;
};

__device__ __forceinline__ SymTile sym_tile_begin(const int4 &H, const double *r, int lane, double (*xs)[TS]) {
  SymTile t;
  t.tile = __builtin_amdgcn_readfirstlane(H.x);
  const int rI = __builtin_amdgcn_readfirstlane(H.y), rJ = __builtin_amdgcn_readfirstlane(H.z);
  const int flags = __builtin_amdgcn_readfirstlane(H.w);
  t.f32 = (flags & 1) != 0;
  t.offd = (flags & 2) != 0;
  const double xi = r[rI + lane], xj = r[rJ + lane];
  // the previous tile's reads of xs are done before it is rewritten
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  xs[0][lane] = xi;
  xs[1][lane] = xj;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  return t;
}

// Row partial A_IJ x_J and, off the diagonal, column partial A_IJ^T x_I of
// every kept tile, one wavefront per tile.  Two forms with the same sums,
// term by term: k_sym_tiles_all issues every load of a tile at once (two
// wavefronts per SIMD), for solves with few tiles per wavefront, where a
// tile's load latency is the cost; k_sym_tiles_stream takes quarters of 8
// loads, the next requested while the current one is summed (four
// wavefronts per SIMD; the tile is found through the kept list and the tile
// table, and x is gathered in dof order), for solves that stream many tiles
// per wavefront.
__global__ __launch_bounds__(256, 2) void k_sym_tiles_all(const double *__restrict__ packed,
                                                       const int4 *__restrict__ hdr, const double *__restrict__ r,
                                                       const int64_t *__restrict__ n_kept,
                                                       double *__restrict__ rowpart, double *__restrict__ colpart) {
  const int64_t n_tiles = *n_kept;
  __shared__ double xs[4][2][TS];  // per wavefront: x_I, x_J
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
  const int h = lane >> 5, c0 = 2 * (lane & 31);
  const int64_t stride = (int64_t)gridDim.x * 4;
  for (int64_t k = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + w)); k < n_tiles; k += stride) {
    const int4 H = hdr[k];
    const double *tp = packed + (int64_t)__builtin_amdgcn_readfirstlane(H.x) * TS * TS;
    const bool f32 = (__builtin_amdgcn_readfirstlane(H.w) & 1) != 0;
    double2 e[32];
#pragma unroll
    for (int qt = 0; qt < 4; qt++) load_pairs(tp, f32, 8 * qt, lane, &e[8 * qt]);
    const SymTile t = sym_tile_begin(H, r, lane, xs[w]);
    const double xj0 = xs[w][1][c0], xj1 = xs[w][1][c0 + 1];
    double cs0 = 0.0, cs1 = 0.0;
#pragma unroll
    for (int qt = 0; qt < 4; qt++) {
      double p[8];
#pragma unroll
      for (int q = 0; q < 8; q++) {
        const double xr = xs[w][0][2 * (8 * qt + q) + h];
        cs0 += e[8 * qt + q].x * xr;
        cs1 += e[8 * qt + q].y * xr;
        p[q] = e[8 * qt + q].x * xj0 + e[8 * qt + q].y * xj1;
      }
      sym_quarter_rows(p, lane, qt, rowpart + t.tile * TS);
    }
    cs0 += __shfl_xor(cs0, 32, WAVE);
    cs1 += __shfl_xor(cs1, 32, WAVE);
    if (t.offd && h == 0) *reinterpret_cast<double2 *>(colpart + t.tile * TS + c0) = double2{cs0, cs1};
  }
}

__global__ __launch_bounds__(256, 4) void k_sym_tiles_stream(const double *packed, const int32_t *tile_meta,
                                                          const int64_t *off, const int32_t *idx, const double *r,
                                                          const int32_t *kept, const uint8_t *kept_f32,
                                                          const int64_t *n_kept, double *rowpart, double *colpart) {
  const int64_t n_tiles = *n_kept;
  __shared__ double xs[4][2][TS];  // per wavefront: x_I, x_J
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
  const int h = lane >> 5, c0 = 2 * (lane & 31);
  const bool b4 = (lane >> 4) & 1, b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1;
  const int64_t stride = (int64_t)gridDim.x * 4;
  for (int64_t k = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + w)); k < n_tiles; k += stride) {
    const int64_t tile = kept[k];
    const bool f32 = __builtin_amdgcn_readfirstlane((int)kept_f32[k]) != 0;
    const double *tp = packed + tile * TS * TS;
    double2 e[8];
    load_pairs(tp, f32, 0, lane, e);
    const int comp = tile_meta[tile * 3 + 0], I = tile_meta[tile * 3 + 1], J = tile_meta[tile * 3 + 2];
    const int64_t base = off[comp], n = off[comp + 1] - base;
    {
      const int64_t gi = (int64_t)I * TS + lane, gj = (int64_t)J * TS + lane;
      const double xi = gi < n ? r[idx[base + gi]] : 0.0;
      const double xj = gj < n ? r[idx[base + gj]] : 0.0;
      // the previous tile's reads of xs are done before it is rewritten
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      xs[w][0][lane] = xi;
      xs[w][1][lane] = xj;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    const double xj0 = xs[w][1][c0], xj1 = xs[w][1][c0 + 1];
    double cs0 = 0.0, cs1 = 0.0;
#pragma unroll 1
    for (int qt = 0; qt < 4; qt++) {  // quarters of 8 loads (16 rows)
      double p[8];
#pragma unroll
      for (int q = 0; q < 8; q++) {
        const double xr = xs[w][0][2 * (8 * qt + q) + h];
        cs0 += e[q].x * xr;
        cs1 += e[q].y * xr;
        p[q] = e[q].x * xj0 + e[q].y * xj1;
      }
      if (qt < 3) load_pairs(tp, f32, 8 * (qt + 1), lane, e);
      // recursive halving over the 32 lanes of the half-wavefront
      double p4[4], p2[2];
#pragma unroll
      for (int kk = 0; kk < 4; kk++)
        p4[kk] = pick(b4, p[kk], p[4 + kk]) + __shfl_xor(pick(b4, p[4 + kk], p[kk]), 16, WAVE);
#pragma unroll
      for (int kk = 0; kk < 2; kk++)
        p2[kk] = pick(b3, p4[kk], p4[2 + kk]) + __shfl_xor(pick(b3, p4[2 + kk], p4[kk]), 8, WAVE);
      double p1 = pick(b2, p2[0], p2[1]) + __shfl_xor(pick(b2, p2[1], p2[0]), 4, WAVE);
      p1 += __shfl_xor(p1, 2, WAVE);
      p1 += __shfl_xor(p1, 1, WAVE);
      // the four lanes 4k .. 4k + 3 of the half hold row 2 (8 qt + k) + h, k = (lane % 32) / 4
      if ((lane & 3) == 0) rowpart[tile * TS + 2 * (8 * qt + ((lane & 31) >> 2)) + h] = p1;
    }
    cs0 += __shfl_xor(cs0, 32, WAVE);
    cs1 += __shfl_xor(cs1, 32, WAVE);
    if (I != J && h == 0) *reinterpret_cast<double2 *>(colpart + tile * TS + c0) = double2{cs0, cs1};
  }
}

// y[idx[i]] = sum_{J <= I} rowpart(I, J) + sum_{J > I} colpart(J, I) over the
// kept tiles of block row I.  One workgroup per block row; wave w takes the
// terms with J = w mod kRedWaves, listed for it in ascending J, and the wave
// sums are added in a fixed order.  (The skipped tiles' partial sums
// are zero, and none of these sums is ever -0, so leaving them out changes no
// bit.)
constexpr int kRedWaves = 16;  // wavefronts per block row in the reduction

__global__ __launch_bounds__(kRedWaves * 64) void k_sym_reduce_list(const int64_t *off, const int32_t *row_comp,
                                                              const int32_t *row_block, const int32_t *idx,
                                                              const int32_t *red_off, const int2 *red,
                                                              const double *rowpart, const double *colpart,
                                                              double *y, double *y2) {
  __shared__ double part[kRedWaves][TS];
  const int64_t c = row_comp[blockIdx.x], I = row_block[blockIdx.x];
  const int64_t n = off[c + 1] - off[c];
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
  double s = 0.0;
  const int e1 = red_off[blockIdx.x * kRedWaves + w + 1];
  for (int e = red_off[blockIdx.x * kRedWaves + w]; e < e1; e++) {
    const int2 E = red[e];
    s += ((E.x & 1) ? colpart : rowpart)[(int64_t)(E.x >> 1) * TS + lane];
  }
  part[w][lane] = s;
  __syncthreads();
  if (w == 0) {
    const int64_t i = I * TS + lane;
    double tot = part[0][lane];
    for (int q = 1; q < kRedWaves; q++) tot += part[q][lane];  // fixed order
    if (i < n) {
      y[idx[off[c] + i]] = tot;
      if (y2) y2[idx[off[c] + i]] = tot;
    }
  }
}

// The same sums for the streaming solve, whose block rows keep most of
// their tiles: wave w walks J = w, w + kRedWaves, .. directly (a skipped
// tile's partial sum is zero).
__global__ __launch_bounds__(kRedWaves * 64) void k_sym_reduce(const int64_t *off, const int64_t *tile_base,
                                                              const int32_t *row_comp, const int32_t *row_block,
                                                              const int32_t *idx, const double *rowpart,
                                                              const double *colpart, double *y, double *y2) {
  __shared__ double part[kRedWaves][TS];
  const int64_t c = row_comp[blockIdx.x], I = row_block[blockIdx.x];
  const int64_t n = off[c + 1] - off[c], T = (n + TS - 1) / TS, tb = tile_base[c];
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
  double s = 0.0;
  for (int64_t k = w; k < T; k += kRedWaves) {
    s += k <= I ? rowpart[(tb + I * (I + 1) / 2 + k) * TS + lane] : colpart[(tb + k * (k + 1) / 2 + I) * TS + lane];
  }
  part[w][lane] = s;
  __syncthreads();
  if (w == 0) {
    const int64_t i = I * TS + lane;
    double tot = part[0][lane];
    for (int q = 1; q < kRedWaves; q++) tot += part[q][lane];  // fixed order
    if (i < n) {
      y[idx[off[c] + i]] = tot;
      if (y2) y2[idx[off[c] + i]] = tot;
    }
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
  {
    const int64_t Tm = (B.n_max + TS - 1) / TS;
    B.pv = ar.alloc<double>((size_t)std::max<int64_t>(Tm, 1) * TS * KB);
    B.pw = ar.alloc<double>((size_t)std::max<int64_t>(Tm, 1) * TS * KB);
    B.pinv = ar.alloc<double>((size_t)TS * TS);
    B.pblk = ar.alloc<double>((size_t)KB * KB);
  }
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
  // right-hand side in component-block order: dof h_idx[h_off[c] + p] sits at
  // pbase[c] + p, component c padded with zeros to whole tiles
  int64_t nr = 0, ndof = 0;
  std::vector<int64_t> pbase(B.n_comp + 1, 0);
  for (int64_t c = 0; c < B.n_comp; c++) {
    pbase[c + 1] = pbase[c] + (B.h_off[c + 1] - B.h_off[c] + TS - 1) / TS * TS;
    for (int64_t q = B.h_off[c]; q < B.h_off[c + 1]; q++) ndof = std::max<int64_t>(ndof, B.h_idx[q] + 1);
  }
  nr = pbase[B.n_comp];
  std::vector<int32_t> rpos((size_t)std::max<int64_t>(ndof, s.nl), -1);
  for (int64_t c = 0; c < B.n_comp; c++)
    for (int64_t q = B.h_off[c]; q < B.h_off[c + 1]; q++) rpos[B.h_idx[q]] = (int32_t)(pbase[c] + q - B.h_off[c]);
  B.rperm = ar.alloc<double>((size_t)std::max<int64_t>(nr, 1));
  B.rpos = ar.alloc<int32_t>(rpos.size());
  B.hdr = ar.alloc<int4>((size_t)std::max<int64_t>(B.n_tiles, 1));
  B.red_off = ar.alloc<int32_t>((size_t)B.n_rows * kRedWaves + 1);
  B.red = ar.alloc<int2>((size_t)std::max<int64_t>(2 * B.n_tiles, 1));
  B.h_pbase = pbase;
  MTS_HIP(hipMemsetAsync(B.rperm, 0, sizeof(double) * (size_t)std::max<int64_t>(nr, 1), st));
  MTS_HIP(hipMemcpyAsync(B.rpos, rpos.data(), sizeof(int32_t) * rpos.size(), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemcpyAsync(B.row_comp, rc.data(), sizeof(int32_t) * rc.size(), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemcpyAsync(B.row_block, rb.data(), sizeof(int32_t) * rb.size(), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemcpyAsync(B.idx, B.h_idx.data(), sizeof(int32_t) * B.h_idx.size(), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemcpyAsync(B.off, B.h_off.data(), sizeof(int64_t) * (B.n_comp + 1), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemcpyAsync(B.tile_meta, meta.data(), sizeof(int32_t) * meta.size(), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemcpyAsync(B.tile_base, tbase.data(), sizeof(int64_t) * (B.n_comp + 1), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemsetAsync(B.colpart, 0, sizeof(double) * B.n_tiles * TS, st));
  MTS_HIP(hipStreamSynchronize(st));
}

// Invert every component block of H (assembled in s.H) in packed lower tiles.
void sym_blocks_build(Solver &s) {
  auto &B = s.sym;
  hipStream_t st = s.stream;
  int64_t tb = 0;
  for (int64_t c = 0; c < B.n_comp; c++) {
    const int64_t n = B.h_off[c + 1] - B.h_off[c];
    const int64_t T = (n + TS - 1) / TS, ntile = T * (T + 1) / 2;
    double *pk = B.packed + tb * TS * TS;
    tb += ntile;
    k_pack_lower<<<(unsigned)((ntile * TS * TS + 255) / 256), 256, 0, st>>>(s.H, s.nl, B.idx + B.h_off[c], n, T, pk);
    MTS_LAUNCH_CHECK();
    for (int64_t k0 = 0; k0 < T; k0 += NB) {
      const int nb = (int)std::min<int64_t>(NB, T - k0);
      // the diagonal block, tile by tile (leaves -A_KK^-1 there)
      for (int64_t k = k0; k < k0 + nb; k++) {
        k_tile_inverse<<<1, 256, 0, st>>>(pk, k, n, B.pinv);
        MTS_LAUNCH_CHECK();
        k_sweep_panel<<<(unsigned)nb, 256, 0, st>>>(pk, k, B.pinv, B.pv, B.pw, k0);
        MTS_LAUNCH_CHECK();
        k_sweep_update<<<(unsigned)(nb * (nb + 1) / 2), 256, 0, st>>>(pk, k, B.pinv, B.pv, B.pw, k0);
        MTS_LAUNCH_CHECK();
      }
      if (nb == T) break;  // one block: done
      // the rest of the matrix, one rank-64 nb update
      k_pblock<<<(unsigned)((nb * TS * nb * TS + 255) / 256), 256, 0, st>>>(pk, k0, nb, B.pblk);
      MTS_LAUNCH_CHECK();
      k_block_panel<<<dim3((unsigned)T, (unsigned)nb), 256, 0, st>>>(pk, k0, nb, B.pblk, B.pv, B.pw);
      MTS_LAUNCH_CHECK();
      k_block_update<<<(unsigned)ntile, 256, 0, st>>>(pk, k0, nb, B.pv, B.pw);
      MTS_LAUNCH_CHECK();
    }
    // the sweep leaves -H^-1
    k_negate<<<(unsigned)((ntile * TS * TS + 255) / 256), 256, 0, st>>>(pk, ntile * TS * TS);
    MTS_LAUNCH_CHECK();
    vlog(s, "coupling: block %lld of %lld inverted (%lld dofs)", (long long)(c + 1), (long long)B.n_comp,
         (long long)n);
  }
  sym_blocks_prune(s);
}

// The tiles each multiplier solve reads.  The inverse of H decays
// exponentially with the distance between constraints (H couples constraints
// within twice the response reach); a tile whose largest entry is at most
// kInvDrop of the largest entry of its component adds at most
// (dofs) x kInvDrop x max|H^-1| x max|r| to any multiplier, far below the
// rounding of the product itself (dofs x eps relative), so it is skipped.
// Skipped tiles keep zero partial sums, so the fixed-order reduction is
// unchanged.  A kept tile whose largest entry is at most 2^-29 of its
// component's largest is stored in FP32: rounding then moves an entry by at
// most 2^-54 of the component's largest entry, half a unit in the last place
// of that entry in FP64, and the products and sums stay in FP64 in the same
// order.  MTS_INV_DROP=0 keeps every tile, in FP64.
void sym_blocks_prune(Solver &s) {
  constexpr double kInvDrop = 1e-18;
  const double kF32 = std::ldexp(1.0, -29);
  auto &B = s.sym;
  hipStream_t st = s.stream;
  if (!B.n_tiles) return;
  if (!B.tile_max) B.tile_max = s.arena.alloc<double>((size_t)B.n_tiles);
  if (!B.kept) B.kept = s.arena.alloc<int32_t>((size_t)B.n_tiles);
  if (!B.n_kept_dev) B.n_kept_dev = s.arena.alloc<int64_t>(1);
  k_tile_absmax<<<(unsigned)B.n_tiles, WAVE, 0, st>>>(B.packed, B.n_tiles, B.tile_max);
  MTS_LAUNCH_CHECK();
  std::vector<double> tm((size_t)B.n_tiles);
  std::vector<int32_t> meta((size_t)B.n_tiles * 3);
  MTS_HIP(hipMemcpyAsync(tm.data(), B.tile_max, sizeof(double) * tm.size(), hipMemcpyDeviceToHost, st));
  MTS_HIP(hipMemcpyAsync(meta.data(), B.tile_meta, sizeof(int32_t) * meta.size(), hipMemcpyDeviceToHost, st));
  MTS_HIP(hipStreamSynchronize(st));
  std::vector<double> cmax((size_t)B.n_comp, 0.0);
  for (int64_t t = 0; t < B.n_tiles; t++) cmax[meta[t * 3]] = std::max(cmax[meta[t * 3]], tm[t]);
  std::vector<int32_t> kept, to32;
  std::vector<uint8_t> f32;
  for (int64_t t = 0; t < B.n_tiles; t++) {
    const double cm = cmax[meta[t * 3]];
    const bool diag = meta[t * 3 + 1] == meta[t * 3 + 2];
    if (!B.prune || diag || tm[t] > kInvDrop * cm) {
      kept.push_back((int32_t)t);
      // FP32 only in its normal range (no subnormal entries above the drop)
      const bool low = B.prune && !diag && tm[t] <= kF32 * cm && kInvDrop * cm >= 1e-30 && cm <= 1e30;
      f32.push_back(low ? 1 : 0);
      if (low) to32.push_back((int32_t)t);
    }
  }
  B.n_kept = (int64_t)kept.size();
  B.n_kept32 = (int64_t)to32.size();
  {
    // kept-tile headers, and per block row its kept partial sums in
    // ascending block column (the zero partials of skipped tiles add nothing)
    std::vector<int64_t> rowbase(B.n_comp + 1, 0);
    for (int64_t c = 0; c < B.n_comp; c++)
      rowbase[c + 1] = rowbase[c] + (B.h_off[c + 1] - B.h_off[c] + TS - 1) / TS;
    std::vector<int4> hdr(kept.size());
    // one list per block row and reduction wavefront (block column mod kRedWaves)
    std::vector<std::vector<int2>> per_row((size_t)B.n_rows * kRedWaves);
    for (size_t q = 0; q < kept.size(); q++) {
      const int32_t t = kept[q];
      const int32_t c = meta[(size_t)t * 3], I = meta[(size_t)t * 3 + 1], J = meta[(size_t)t * 3 + 2];
      hdr[q] = int4{t, (int32_t)(B.h_pbase[c] + (int64_t)I * TS), (int32_t)(B.h_pbase[c] + (int64_t)J * TS),
                    (f32[q] ? 1 : 0) | (I != J ? 2 : 0)};
      per_row[(size_t)(rowbase[c] + I) * kRedWaves + J % kRedWaves].push_back(int2{t * 2, J});
      if (I != J) per_row[(size_t)(rowbase[c] + J) * kRedWaves + I % kRedWaves].push_back(int2{t * 2 + 1, I});
    }
    std::vector<int32_t> roff(1, 0);
    std::vector<int2> red;
    for (auto &v : per_row) {
      std::sort(v.begin(), v.end(), [](const int2 &a, const int2 &b) { return a.y < b.y; });
      red.insert(red.end(), v.begin(), v.end());
      roff.push_back((int32_t)red.size());
    }
    MTS_HIP(hipMemcpyAsync(B.hdr, hdr.data(), sizeof(int4) * hdr.size(), hipMemcpyHostToDevice, st));
    MTS_HIP(hipMemcpyAsync(B.red_off, roff.data(), sizeof(int32_t) * roff.size(), hipMemcpyHostToDevice, st));
    MTS_HIP(hipMemcpyAsync(B.red, red.data(), sizeof(int2) * red.size(), hipMemcpyHostToDevice, st));
    MTS_HIP(hipStreamSynchronize(st));  // before the host vectors go away
  }
  if (!B.kept_f32) B.kept_f32 = s.arena.alloc<uint8_t>((size_t)B.n_tiles);
  MTS_HIP(hipMemcpyAsync(B.kept, kept.data(), sizeof(int32_t) * kept.size(), hipMemcpyHostToDevice, st));
  MTS_HIP(hipMemcpyAsync(B.kept_f32, f32.data(), f32.size(), hipMemcpyHostToDevice, st));
  if (!to32.empty()) {
    int32_t *d32 = s.arena.alloc<int32_t>(to32.size());
    MTS_HIP(hipMemcpyAsync(d32, to32.data(), sizeof(int32_t) * to32.size(), hipMemcpyHostToDevice, st));
    k_tiles_to_f32<<<(unsigned)to32.size(), 256, 0, st>>>(B.packed, d32);
    MTS_LAUNCH_CHECK();
    MTS_HIP(hipStreamSynchronize(st));
    s.arena.release(d32);
  }
  MTS_HIP(hipMemcpyAsync(B.n_kept_dev, &B.n_kept, sizeof(int64_t), hipMemcpyHostToDevice, st));
  // skipped tiles contribute zero partial sums
  MTS_HIP(hipMemsetAsync(B.rowpart, 0, sizeof(double) * B.n_tiles * TS, st));
  MTS_HIP(hipMemsetAsync(B.colpart, 0, sizeof(double) * B.n_tiles * TS, st));
  MTS_HIP(hipStreamSynchronize(st));
  vlog(s, "coupling: the multiplier solve reads %lld of %lld tiles (%lld in FP32)", (long long)B.n_kept,
       (long long)B.n_tiles, (long long)B.n_kept32);
}

// Kept tiles up to which a solve issues every load of a tile at once and
// reduces over lists of its kept tiles (about two tiles per resident
// wavefront: 2048 at two per SIMD on 256 CUs); above it the solve streams
// quarters of tiles and reduces over every tile of a block row.  Both forms
// give the same bits for any count, so a solve captured in a graph stays
// valid when a rebuild moves the count across this bound.
constexpr int64_t kSymFullTiles = 4096;

void sym_blocks_apply(Solver &s, const double *r_dof, const double *r_blk, double *y, double *y2) {
  auto &B = s.sym;
  if (!B.n_tiles) return;
  // four tiles per workgroup at a time; up to eight resident workgroups per CU
  // the grid covers every tile; the count of kept tiles is read on the device
  const unsigned g = (unsigned)std::min<int64_t>((B.n_tiles + 3) / 4, 256 * 8);
  if (B.form == 1 || (B.form == 0 && B.n_kept <= kSymFullTiles)) {
    k_sym_tiles_all<<<g, 256, 0, s.stream>>>(B.packed, B.hdr, r_blk, B.n_kept_dev, B.rowpart, B.colpart);
    MTS_LAUNCH_CHECK();
    k_sym_reduce_list<<<(unsigned)B.n_rows, kRedWaves * 64, 0, s.stream>>>(
        B.off, B.row_comp, B.row_block, B.idx, B.red_off, B.red, B.rowpart, B.colpart, y, y2);
  } else {
    k_sym_tiles_stream<<<g, 256, 0, s.stream>>>(B.packed, B.tile_meta, B.off, B.idx, r_dof, B.kept, B.kept_f32,
                                                B.n_kept_dev, B.rowpart, B.colpart);
    MTS_LAUNCH_CHECK();
    k_sym_reduce<<<(unsigned)B.n_rows, kRedWaves * 64, 0, s.stream>>>(B.off, B.tile_base, B.row_comp, B.row_block,
                                                                      B.idx, B.rowpart, B.colpart, y, y2);
  }
  MTS_LAUNCH_CHECK();
}

}  // namespace mts
