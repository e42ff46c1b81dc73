// Dense FP64 linear algebra for the multiplier system of Eq. 49: the symmetric
// positive-definite matrix H is inverted once per (re)build by blocked in-place
// Gauss-Jordan elimination (no pivoting, SPD), and every macro step applies
// the inverse with a row-per-wavefront GEMV.
#include "internal.h"

namespace mts {

namespace {

constexpr int NB = 64;

// Invert the kb x kb pivot block A[k0:k0+kb, k0:k0+kb] in LDS (Gauss-Jordan).
__global__ __launch_bounds__(256) void k_pivot_inverse(const double *A, int64_t n, int64_t k0, int kb,
                                                      double *pinv) {
  __shared__ double M[NB][NB + 1];
  __shared__ double rowp[NB], colp[NB];
  for (int t = threadIdx.x; t < kb * kb; t += blockDim.x) {
    int r = t / kb, c = t % kb;
    M[r][c] = A[(k0 + r) * n + k0 + c];
  }
  __syncthreads();
  for (int p = 0; p < kb; p++) {
    double d = 1.0 / M[p][p];
    __syncthreads();
    for (int t = threadIdx.x; t < kb; t += blockDim.x) {
      rowp[t] = (t == p) ? d : M[p][t] * d;
      colp[t] = M[t][p];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kb * kb; t += blockDim.x) {
      int r = t / kb, c = t % kb;
      if (r == p) M[r][c] = rowp[c];
      else if (c == p) M[r][c] = -colp[r] * d;
      else M[r][c] = M[r][c] - colp[r] * rowp[c];
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < kb * kb; t += blockDim.x) pinv[t] = M[t / kb][t % kb];
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

// A -= C R over the whole matrix; 64x64 output tile per workgroup, 4x4 per thread.
__global__ __launch_bounds__(256) void k_rank_update(double *A, int64_t n, int kb, const double *C,
                                                     const double *R) {
  __shared__ double Cs[NB][NB + 1];
  __shared__ double Rs[NB][NB + 1];
  int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
  int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  for (int t = threadIdx.x; t < 64 * NB; t += 256) {
    int r = t / NB, c = t % NB;
    int64_t i = i0 + r;
    Cs[r][c] = (i < n && c < kb) ? C[i * kb + c] : 0.0;
    int rr = t / 64, cc = t % 64;
    int64_t j = j0 + cc;
    Rs[rr][cc] = (rr < kb && j < n) ? R[(int64_t)rr * n + j] : 0.0;
  }
  __syncthreads();
  double acc[4][4] = {};
  for (int s = 0; s < kb; s++) {
    double cv[4], rv[4];
    for (int q = 0; q < 4; q++) {
      cv[q] = Cs[ty * 4 + q][s];
      rv[q] = Rs[s][tx * 4 + q];
    }
    for (int a = 0; a < 4; a++)
      for (int b = 0; b < 4; b++) acc[a][b] += cv[a] * rv[b];
  }
  for (int a = 0; a < 4; a++) {
    int64_t i = i0 + ty * 4 + a;
    if (i >= n) continue;
    for (int b = 0; b < 4; b++) {
      int64_t j = j0 + tx * 4 + b;
      if (j < n) A[i * n + j] -= acc[a][b];
    }
  }
}

__global__ __launch_bounds__(256) void k_gemv(const double *A, const double *x, double *y, int64_t n) {
  int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  int lane = threadIdx.x & (WAVE - 1);
  if (row >= n) return;
  const double *a = A + row * n;
  double s = 0.0;
  for (int64_t j = lane; j < n; j += WAVE) s += a[j] * x[j];
  for (int off = WAVE / 2; off > 0; off >>= 1) s += __shfl_down(s, off, WAVE);
  if (lane == 0) y[row] = s;
}

}  // namespace

void dense_spd_inverse(Solver &s, double *A, int64_t n) {
  hipStream_t st = s.stream;
  if (n <= 0) return;
  if (!s.tmpA) {
    s.tmpA = s.arena.alloc<double>((size_t)n * NB);
    s.tmpB = s.arena.alloc<double>((size_t)n * NB);
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

void dense_gemv(hipStream_t st, const double *A, const double *x, double *y, int64_t n) {
  if (n <= 0) return;
  unsigned grid = (unsigned)((n * WAVE + 255) / 256);
  k_gemv<<<grid, 256, 0, st>>>(A, x, y, n);
  MTS_LAUNCH_CHECK();
}

}  // namespace mts
