// Small dense FP64 linear algebra out of LDS.
//
// The reduced Newton systems of the ROM step (r x r, r <= 64: the Galerkin
// system I - dt Phi^T J_f Phi, or the hyper-reduced Gauss-Newton system) are
// solved by LU with partial pivoting.  The pivot search is a wave-wide argmax
// (butterfly of shuffles; on equal magnitudes the lowest row index wins, as
// LAPACK's idamax does), and the back substitution is column-oriented (x_i is
// broadcast, lanes j < i subtract their share).
#pragma once
#include "internal.h"

namespace romhip {

__device__ __forceinline__ void lds_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Solve A x = b in place (b <- x), n <= 64, by LU with partial pivoting run
// by a whole workgroup (any blockDim.x that is a multiple of 64): wave 0 finds the pivot, the row swap and the
// trailing update of the augmented system [A | b] are spread over all
// threads (right-looking elimination, three barriers per column), and wave 0
// back-substitutes.  A (row-major, leading dimension ld) and b live in LDS;
// b <- x.  Returns 1, or 0 after a zero pivot.  All threads must call it.
__device__ inline int block_lu_solve(double* A, int ld, double* b, int n) {
  __shared__ int piv;
  __shared__ int okf;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) okf = 1;
  for (int k = 0; k < n; ++k) {
    if (tid < 64) {
      const double a = (tid >= k && tid < n) ? fabs(A[tid * ld + k]) : -1.0;
      // the lowest lane holding the largest |a| (NaN entries are never chosen
      // over numbers; an all-NaN column takes the lowest candidate row)
      const double key = isnan(a) ? -0.5 : a;
      const double v = wave_max_bfly(key);
      const int idx = (int)__builtin_ctzll(__ballot(key == v));
      if (tid == 0) {
        piv = idx;
        if (v == 0.0) okf = 0;
      }
    }
    __syncthreads();
    const int p = piv;
    if (p != k) {
      for (int j = tid; j < n; j += nt) {
        const double t = A[k * ld + j];
        A[k * ld + j] = A[p * ld + j];
        A[p * ld + j] = t;
      }
      if (tid == 0) { const double t = b[k]; b[k] = b[p]; b[p] = t; }
    }
    __syncthreads();
    const double pk = A[k * ld + k];
    const double ipk = pk != 0.0 ? 1.0 / pk : 0.0;
    const int rows = n - k - 1, cols = n - k;  // column n - k - 1 of the update is b
    for (int e = tid; e < rows * cols; e += nt) {
      const int i = k + 1 + e / cols, jj = e % cols;
      const double f = A[i * ld + k] * ipk;
      if (jj < cols - 1) A[i * ld + k + 1 + jj] -= f * A[k * ld + k + 1 + jj];
      else b[i] -= f * b[k];
    }
    __syncthreads();
  }
  if (tid < 64) {
    for (int i = n - 1; i >= 0; --i) {
      const double d = A[i * ld + i];
      const double xi = d != 0.0 ? b[i] / d : 0.0;
      if (tid < i) b[tid] -= A[tid * ld + i] * xi;
      if (tid == i) b[i] = xi;
      lds_wave_sync();
    }
  }
  __syncthreads();
  return okf;
}

}  // namespace romhip
