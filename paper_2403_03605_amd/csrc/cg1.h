// One-right-hand-side Jacobi-preconditioned conjugate gradients (x <- A^-1 b)
// in three launches per iteration: the caller's operator (q = A p, with
// per-workgroup partial sums of p.q), the update of x, r and z (with partial
// sums of the new r.z) and the new direction.  Dot products keep a fixed
// order: per-workgroup tree sums of the products, then a strided sum over the
// workgroups and a tree over the threads, which every workgroup that needs the
// total recomputes for itself (the same sum in the same order, so every
// workgroup gets the same value).  A device flag ends the iterations once
// r.z <= tol r0.z0 (after at least kCgMinIters): the kernels of later
// iterations return at once.  Used by the implicit FE and PD steps.
#pragma once

#include "internal.h"

#include <algorithm>

namespace mts {

namespace {

constexpr int kCgT = 256;  // threads per workgroup of the vector kernels

// At least this many iterations per solve: where the step is small A is
// nearly its diagonal and r.z falls below the tolerance after one or two
// iterations while dofs of small weighted mass (near the PD-only box) still
// carry a relative error of 1e-4; eight iterations bring them to rounding.
constexpr int kCgMinIters = 8;

struct Cg1 {
  int64_t ndof, nblk;  // vector length; workgroups of the vector kernels (kCgT threads)
  int64_t nblk_pq;     // partial sums of p.q the operator writes
  const double *inv_diag;
  double *x, *r, *z, *p, *q;
  double *part_pq, *part_rz0, *part_rz[2];
  int32_t *state;  // [0] done, [1] iterations run
  double tol;
};

__device__ inline double block_tree(double v, double *lds) {
  lds[threadIdx.x] = v;
  __syncthreads();
  for (int h = kCgT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) lds[threadIdx.x] += lds[threadIdx.x + h];
    __syncthreads();
  }
  const double out = lds[0];
  __syncthreads();
  return out;
}

__device__ inline double total_of(const double *part, int64_t nblk, double *lds) {
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < nblk; k += kCgT) s += part[k];
  return block_tree(s, lds);
}

// x = 0, r = b, z = p = D^-1 b, partial sums of r.z; clears the flag
__global__ __launch_bounds__(kCgT) void k_cg1_init(Cg1 C, const double *b) {
  __shared__ double lds[kCgT];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (t < C.ndof) {
    const double zi = b[t] * C.inv_diag[t];
    C.x[t] = 0.0;
    C.r[t] = b[t];
    C.z[t] = zi;
    C.p[t] = zi;
    v = b[t] * zi;
  }
  const double sum = block_tree(v, lds);
  if (threadIdx.x == 0) {
    C.part_rz0[blockIdx.x] = sum;
    C.part_rz[0][blockIdx.x] = sum;
    if (blockIdx.x == 0) {
      C.state[0] = 0;
      C.state[1] = 0;
    }
  }
}

// x += alpha p, r -= alpha q, z = D^-1 r, partial sums of the new r.z
__global__ __launch_bounds__(kCgT) void k_cg1_step(Cg1 C, int cur) {
  __shared__ double lds[kCgT];
  if (C.state[0]) return;
  const double pq = total_of(C.part_pq, C.nblk_pq, lds);
  const double rz = total_of(C.part_rz[cur], C.nblk, lds);
  const double al = pq > 0.0 ? rz / pq : 0.0;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (t < C.ndof) {
    C.x[t] = C.x[t] + al * C.p[t];
    const double rn = C.r[t] - al * C.q[t];
    C.r[t] = rn;
    const double zn = rn * C.inv_diag[t];
    C.z[t] = zn;
    v = rn * zn;
  }
  const double sum = block_tree(v, lds);
  if (threadIdx.x == 0) C.part_rz[cur ^ 1][blockIdx.x] = sum;
}

// p = z + beta p; the flag once r.z <= tol r0.z0
__global__ __launch_bounds__(kCgT) void k_cg1_dir(Cg1 C, int cur) {
  __shared__ double lds[kCgT];
  if (C.state[0]) return;
  const double rzn = total_of(C.part_rz[cur ^ 1], C.nblk, lds);
  const double rzo = total_of(C.part_rz[cur], C.nblk, lds);
  const double be = rzo > 0.0 ? rzn / rzo : 0.0;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < C.ndof) C.p[t] = C.z[t] + be * C.p[t];
  if (blockIdx.x == 0) {
    const double rz0 = total_of(C.part_rz0, C.nblk, lds);
    if (threadIdx.x == 0) {
      const int done_its = C.state[1] + 1;
      C.state[1] = done_its;
      if (done_its >= kCgMinIters && rzn <= C.tol * rz0) C.state[0] = 1;
    }
  }
}

// Runs the iterations on C from x = 0 (b given) with apply() launching the
// operator for the current direction; the host reads the flag after as many
// iterations as the previous solve needed plus one (at least kCgMinIters),
// then every eight.  Returns the iterations run.
template <class Apply>
int64_t cg1_run(hipStream_t st, const Cg1 &C, const double *b, int64_t iters_last, int32_t *h_state, Apply apply) {
  const unsigned g = (unsigned)C.nblk;
  k_cg1_init<<<g, kCgT, 0, st>>>(C, b);
  MTS_LAUNCH_CHECK();
  int cur = 0;
  int64_t it = 0, batch = std::max<int64_t>(kCgMinIters, iters_last + 1);
  const int64_t max_it = 4000;
  for (;;) {
    for (int64_t k = 0; k < batch; k++, it++) {
      apply();
      k_cg1_step<<<g, kCgT, 0, st>>>(C, cur);
      MTS_LAUNCH_CHECK();
      k_cg1_dir<<<g, kCgT, 0, st>>>(C, cur);
      MTS_LAUNCH_CHECK();
      cur ^= 1;
    }
    MTS_HIP(hipMemcpyAsync(h_state, C.state, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    MTS_HIP(hipStreamSynchronize(st));
    if (h_state[0]) break;
    if (it >= max_it) throw ArgError{"conjugate gradients did not converge"};
    batch = 8;
  }
  return h_state[1];
}

}  // namespace

}  // namespace mts
